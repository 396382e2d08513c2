// lrq_device.hip -- gfx950 kernels of the longest-repeat query and the C-ABI
// entry points that launch them.
//
// Method: Y. Tian and B. Xu, "On Longest Repeat Queries Using GPU" (arXiv
// 1501.06663).  0-based positions throughout.  Every kernel is integer,
// memory-bound work (no MFMA): the design goals are coalesced 16-byte
// streaming where the access pattern allows it, one random cache line per
// position where it does not, and wave64 ballots for compaction.
//
// Every index that a kernel derives from its inputs (SA values, neighbour
// indices, segment offsets, compact-array counts, query positions) is checked
// against the sizes the host passed before it is dereferenced, so malformed
// inputs set error bits instead of reading or writing out of bounds.

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "lrq.h"
#include "lrq_internal.h"

namespace lrq {
namespace {

constexpr int WAVE = 64;

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

__device__ __forceinline__ int64_t imin(int64_t a, int64_t b) { return a < b ? a : b; }
__device__ __forceinline__ int64_t imax(int64_t a, int64_t b) { return a > b ? a : b; }

__device__ __forceinline__ void raise_err(uint32_t *err, uint32_t bit) {
    atomicOr(err, bit);
}

// Non-temporal 8-byte pair accesses, for data touched once.
__device__ __forceinline__ int2 load_stream(const int2 *p) {
    const uint64_t q = __builtin_nontemporal_load(reinterpret_cast<const uint64_t *>(p));
    return make_int2(int32_t(uint32_t(q)), int32_t(q >> 32));
}
__device__ __forceinline__ void store_stream(int2 *p, int2 v) {
    __builtin_nontemporal_store((uint64_t(uint32_t(v.y)) << 32) | uint32_t(v.x),
                                reinterpret_cast<uint64_t *>(p));
}

// Positions and lengths have the type P: int32 up to LRQ_MAX_TOTAL, int64
// beyond it (the lrq64_ calls).  A (start, length) record, or the pair of a
// position's two neighbours or two lcp values, is a pair_t<P>.
template <class P> struct PairOf;
template <> struct PairOf<int32_t> { using type = int2; };
template <> struct PairOf<int64_t> { using type = longlong2; };
template <class P> using pair_t = typename PairOf<P>::type;

// Index arithmetic of the LCP compares.  With 32-bit positions every
// position, position + lcp and position + one round of a wave's compare stays
// below 2^32 (positions and lengths are below 2^31), so unsigned 32-bit math
// is exact and cheaper than 64-bit; 64-bit positions keep int64.
template <class P> struct IndexOf;
template <> struct IndexOf<int32_t> { using type = uint32_t; };
template <> struct IndexOf<int64_t> { using type = int64_t; };
template <class P> using ix_t = typename IndexOf<P>::type;

template <class P>
__device__ __forceinline__ pair_t<P> mkpair(P a, P b) {
    pair_t<P> r;
    r.x = a;
    r.y = b;
    return r;
}

typedef long long v2i64 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ longlong2 load_stream(const longlong2 *p) {
    const v2i64 q = __builtin_nontemporal_load(reinterpret_cast<const v2i64 *>(p));
    longlong2 r;
    r.x = q.x;
    r.y = q.y;
    return r;
}
__device__ __forceinline__ void store_stream(longlong2 *p, longlong2 v) {
    const v2i64 q = {v.x, v.y};
    __builtin_nontemporal_store(q, reinterpret_cast<v2i64 *>(p));
}

// ---- segments ---------------------------------------------------------------

// nseg independent strings laid end to end; off == nullptr means one string.
// Offsets are clamped into [0, total] and made non-decreasing on read, so a
// malformed offset array can give wrong answers but never a wild index.
struct Segs {
    const int64_t *off;
    int32_t nseg;
    int64_t total;

    __device__ __forceinline__ int64_t raw(int32_t b) const {
        if (!off) return b <= 0 ? 0 : total;
        int64_t v = off[b];
        return v < 0 ? 0 : (v > total ? total : v);
    }
    __device__ __forceinline__ int64_t begin(int32_t b) const { return raw(b); }
    __device__ __forceinline__ int64_t end(int32_t b) const {
        int64_t e = raw(b + 1), s = raw(b);
        return e < s ? s : e;
    }
    // Largest b in [0, nseg) with begin(b) <= g.
    __device__ __forceinline__ int32_t find(int64_t g) const {
        if (!off) return 0;
        int32_t lo = 0, hi = nseg - 1;
        while (lo < hi) {
            int32_t mid = (lo + hi + 1) >> 1;
            if (raw(mid) <= g) lo = mid; else hi = mid - 1;
        }
        return lo;
    }
    // The same, found by the 64 lanes of a wave together (every lane active,
    // g the same in all): each round probes 64 evenly spaced offsets of the
    // remaining range and keeps the gap after the last one at or below g, so
    // 512 segments take two rounds of loads instead of nine dependent ones.
    __device__ __forceinline__ int32_t find_wave(int64_t g) const {
        if (!off) return 0;
        int32_t lo = 0, hi = nseg - 1;  // the answer is in [lo, hi]
        while (lo < hi) {
            const int32_t step = (hi - lo + WAVE) / WAVE;  // ceil((hi - lo + 1) / 64)
            const int32_t b = lo + lane() * step;
            const bool le = b <= hi && raw(b) <= g;  // true on a prefix of the lanes
            int32_t c = __popcll(__ballot(le));
            c = c > 0 ? c : 1;  // as find: 0 when no begin is at or below g
            lo += (c - 1) * step;
            hi = hi < lo + step - 1 ? hi : lo + step - 1;
        }
        return lo;
    }
    // Advance b until g < end(b).
    __device__ __forceinline__ int32_t advance(int32_t b, int64_t g) const {
        while (b + 1 < nseg && end(b) <= g) ++b;
        return b;
    }
};

// A lane's current segment and its bounds, moved on only when a position
// passes the segment's end: for increasing positions one compare each instead
// of reloading the offsets.
struct SegRun {
    int32_t b;
    int64_t sb, se;
    __device__ __forceinline__ void init(const Segs &segs, int32_t b0, int64_t g) {
        b = segs.advance(b0, g);
        sb = segs.begin(b);
        se = segs.end(b);
    }
    __device__ __forceinline__ void at(const Segs &segs, int64_t g) {
        if (g < se) return;
        b = segs.advance(b, g);
        sb = segs.begin(b);
        se = segs.end(b);
    }
};

// The run of g's segment (as SegRun::init from Segs::find_wave), found by
// the 64 lanes of a wave together (every lane active, g the same in all).  The
// last round of the search probes consecutive starts, one past the range too,
// so the segment's bounds come from the probes themselves and cost no further
// round of loads (unless the range fills all 64 lanes and the answer is its
// last start).
__device__ __forceinline__ SegRun find_run_wave(const Segs &segs, int64_t g) {
    if (!segs.off) return SegRun{0, 0, segs.total};
    int32_t lo = 0, hi = segs.nseg - 1;  // the answer is in [lo, hi]
    for (;;) {
        const int32_t step = (hi - lo + WAVE) / WAVE;  // ceil((hi - lo + 1) / 64)
        const int32_t b = lo + lane() * step;
        // offsets hold nseg + 1 entries, so b = hi + 1 <= nseg is readable
        const bool probe = step == 1 ? b <= hi + 1 : b <= hi;
        const int64_t v = probe ? segs.raw(b) : 0;
        int32_t c = __popcll(__ballot(b <= hi && v <= g));  // true on a prefix of the lanes
        c = c > 0 ? c : 1;  // as find: 0 when no start is at or below g
        if (step == 1) {
            const int32_t r = lo + c - 1;
            const int64_t sb = __shfl(v, c - 1);
            int64_t nx = __shfl(v, c < WAVE ? c : WAVE - 1);  // raw(r + 1), probed by lane c
            if (c == WAVE) nx = segs.raw(r + 1);
            return SegRun{r, sb, nx > sb ? nx : sb};
        }
        lo += (c - 1) * step;
        hi = hi < lo + step - 1 ? hi : lo + step - 1;
    }
}

// ---- text access --------------------------------------------------------------
//
// The LCP kernels only test characters for equality, so they may read the
// text through any one-to-one code.  A text with at most 16 distinct byte
// values is packed to 1, 2 or 4 bits per character (2^lg bits), LSB-first in
// 64-bit words: a 2^24-character DNA text then takes 4 MiB, about the L2 of
// one XCD, instead of 16 MiB, and the random neighbour-side reads of the LCP
// walk mostly hit in L2.  Other texts are read as bytes (lg = 3) straight from
// the caller's buffer.

struct Sym {
    const uint64_t *w;   // packed words, or the text itself when lg == 3
    const uint8_t *b8;   // the text
    int64_t total;
    int64_t nwords;      // words of w that may be read
    int lg;

    __device__ __forceinline__ int per() const { return 64 >> lg; }

    // Characters p .. p + per() - 1, character p in the low bits.  Characters
    // at or past `total` read as 0 or as padding; every compare is clamped to
    // its string's end before it looks at them.
    template <class IX>
    __device__ __forceinline__ uint64_t at(IX p) const {
        const IX a = p >> (6 - lg);                        // word of character p
        const int sh = int(p & IX((64 >> lg) - 1)) << lg;  // its bit offset
        if (a + IX(2) <= IX(nwords)) {  // nwords < 2^32 whenever IX is 32-bit
            const uint64_t lo = w[a];
            if (sh == 0) return lo;
            return (lo >> sh) | (w[a + 1] << (64 - sh));
        }
        return tail(int64_t(p));
    }

    __device__ uint64_t tail(int64_t p) const {
        uint64_t v = 0;
        const int n = per();
        if (lg == 3) {
            for (int q = 0; q < n; ++q)
                if (p + q < total) v |= uint64_t(b8[p + q]) << (8 * q);
        } else {
            const uint64_t m = (uint64_t(1) << (1 << lg)) - 1;
            for (int q = 0; q < n; ++q) {
                const int64_t x = (p + q) << lg;
                if (p + q < total) v |= ((w[x >> 6] >> (x & 63)) & m) << (q << lg);
            }
        }
        return v;
    }

    // Word k of the packed layout; for bytes, text[8k .. 8k+8) with zeros past
    // the end.
    __device__ __forceinline__ uint64_t word(int64_t k) const {
        if (lg != 3) return k < nwords ? w[k] : 0;
        if ((k + 1) * 8 <= total) return w[k];
        return tail(k * 8);
    }
};

__device__ __forceinline__ Sym make_sym(const uint8_t *text, int64_t total, const uint64_t *packed,
                                        int64_t pwords, const int32_t *lgp) {
    Sym g;
    g.b8 = text;
    g.total = total;
    g.lg = *lgp & 3;  // 0..3 whatever the word holds: every read stays in its buffer
    if (g.lg == 3) {
        g.w = reinterpret_cast<const uint64_t *>(text);
        g.nwords = total >> 3;
    } else {
        g.w = packed;
        g.nwords = pwords;
    }
    return g;
}

// Byte values present in the text, ORed into mask[0..8) (cleared beforehand).
__global__ __launch_bounds__(1024) void alpha_kernel(const uint8_t *__restrict__ text, int64_t total,
                                                     uint32_t *mask) {
    uint32_t m[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    auto add = [&](uint32_t c) {
        const uint32_t bit = 1u << (c & 31), k = c >> 5;
#pragma unroll
        for (int q = 0; q < 8; ++q) m[q] |= k == uint32_t(q) ? bit : 0u;
    };
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    const int64_t g0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t *t8 = reinterpret_cast<const uint64_t *>(text);
    const int64_t nw = total >> 3;
    // A word whose eight bytes share their top three bits (so their bits fall
    // in one mask word, as for the letters of a DNA text) sets them in `hot`
    // with one shift and OR per byte; the top bits are those of the thread's
    // first word.  Other words take the general path byte by byte.
    constexpr uint64_t TOP3 = 0xe0e0e0e0e0e0e0e0ull;
    const uint64_t hot_top = g0 < nw ? (t8[g0] & 0xe0u) * 0x0101010101010101ull : 0;
    uint32_t hot = 0;
    for (int64_t k = g0; k < nw; k += 4 * stride) {
        uint64_t v[4];  // four independent loads in flight
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = k + u * stride < nw ? t8[k + u * stride] : 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (k + u * stride >= nw) break;
            if ((v[u] & TOP3) == hot_top) {
#pragma unroll
                for (int q = 0; q < 8; ++q) hot |= 1u << (uint32_t(v[u] >> (8 * q)) & 31u);
            } else {
#pragma unroll
                for (int q = 0; q < 8; ++q) add(uint32_t(v[u] >> (8 * q)) & 255u);
            }
        }
    }
    {
        const uint32_t k = uint32_t(hot_top & 0xe0u) >> 5;
#pragma unroll
        for (int q = 0; q < 8; ++q) m[q] |= k == uint32_t(q) ? hot : 0u;
    }
    for (int64_t p = (total & ~int64_t(7)) + g0; p < total; p += stride) add(text[p]);
    // wave, then block, then one global atomic per new bit word: every block
    // sees the same few values, so most find their bits already set
    __shared__ uint32_t s_m[8];
    if (threadIdx.x < 8) s_m[threadIdx.x] = 0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        uint32_t v = m[q];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
        if (lane() == 0 && v) atomicOr(&s_m[q], v);
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        const uint32_t v = s_m[threadIdx.x];
        if (v) {
            const uint32_t cur = __hip_atomic_load(&mask[threadIdx.x], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
            if (v & ~cur) atomicOr(&mask[threadIdx.x], v);
        }
    }
}

// The code (rank of a byte value among those present), the width, and the
// packed words.  Every block derives the same code from the mask; block 0
// publishes the width.  With more than 16 values nothing is packed.
__global__ __launch_bounds__(256) void pack_kernel(const uint8_t *__restrict__ text, int64_t total,
                                                   const uint32_t *__restrict__ mask,
                                                   uint64_t *__restrict__ packed, int64_t pwords,
                                                   int32_t *lg_out) {
    __shared__ uint8_t code[256];
    __shared__ int32_t s_lg;
    const int t = threadIdx.x;
    {
        const int c = t;  // blockDim.x == 256
        int32_t below = 0;
        for (int q = 0; q < (c >> 5); ++q) below += __popc(mask[q]);
        below += __popc(mask[c >> 5] & ((1u << (c & 31)) - 1u));
        code[c] = uint8_t(below);
    }
    if (t == 0) {
        int32_t sigma = 0;
        for (int q = 0; q < 8; ++q) sigma += __popc(mask[q]);
        const int32_t lg = sigma <= 2 ? 0 : sigma <= 4 ? 1 : sigma <= 16 ? 2 : 3;
        s_lg = lg;
        if (blockIdx.x == 0) *lg_out = lg;
    }
    __syncthreads();
    const int lg = s_lg;
    if (lg == 3) return;
    const int per = 64 >> lg;  // 16, 32 or 64 characters, a multiple of 8
    const uint64_t *t8 = reinterpret_cast<const uint64_t *>(text);
    // Output words whose characters all lie in the text take an unrolled
    // path: every input word, then every code, is loaded before any is used
    // (the general loop below waits for each load and each code lookup in
    // turn).
    auto full = [&](auto PER) {
        constexpr int PC = decltype(PER)::value;  // characters per output word
        constexpr int NW = PC / 8, LG = PC == 16 ? 2 : (PC == 32 ? 1 : 0);
        for (int64_t k = int64_t(blockIdx.x) * blockDim.x + t; k < pwords;
             k += int64_t(gridDim.x) * blockDim.x) {
            const int64_t p0 = k * PC;
            if (p0 + PC > total) continue;  // the tail word: the general loop
            uint64_t in[NW];
#pragma unroll
            for (int u = 0; u < NW; ++u) in[u] = t8[(p0 >> 3) + u];
            uint8_t c[PC];
#pragma unroll
            for (int q = 0; q < PC; ++q) c[q] = code[(in[q >> 3] >> (8 * (q & 7))) & 255u];
            uint64_t v = 0;
#pragma unroll
            for (int q = 0; q < PC; ++q) v |= uint64_t(c[q]) << (q << LG);
            packed[k] = v;
        }
    };
    if (lg == 2) full(std::integral_constant<int, 16>{});
    else if (lg == 1) full(std::integral_constant<int, 32>{});
    else full(std::integral_constant<int, 64>{});
    for (int64_t k = int64_t(blockIdx.x) * blockDim.x + t; k < pwords;
         k += int64_t(gridDim.x) * blockDim.x) {
        const int64_t p0 = k * per;
        if (p0 + per <= total) continue;  // written above
        uint64_t v = 0;
        for (int u = 0; u < per / 8; ++u) {
            const int64_t p = p0 + 8 * u;
            uint64_t bytes;
            int n = 8;
            if (p + 8 <= total) {
                bytes = t8[p >> 3];
            } else {
                bytes = 0;
                n = p < total ? int(total - p) : 0;
                for (int q = 0; q < n; ++q) bytes |= uint64_t(text[p + q]) << (8 * q);
            }
            for (int q = 0; q < n; ++q)
                v |= uint64_t(code[(bytes >> (8 * q)) & 255u]) << ((8 * u + q) << lg);
        }
        packed[k] = v;
    }
}

// The i-side of a compare reads through an LDS copy of the block's text range
// when the two words it needs lie inside it.
struct StagedSym {
    Sym g;
    const uint64_t *lds;  // lds[w] = word ((base << lg) >> 6) + w of the layout
    int64_t base;         // first staged character, a multiple of 64
    int64_t len;          // characters staged

    template <class IX>
    __device__ __forceinline__ uint64_t at(IX p) const {
        // r wraps to a large value for p < base when IX is unsigned, which
        // the upper bound rejects as well
        const IX r = p - IX(base);
        if (r >= 0 && r <= IX(len - 2 * g.per())) {
            const uint32_t r32 = uint32_t(r);
            const uint32_t wi = r32 >> (6 - g.lg);
            const int sh = int(r32 & uint32_t(g.per() - 1)) << g.lg;
            const uint64_t lo = lds[wi];
            if (sh == 0) return lo;
            return (lo >> sh) | (lds[wi + 1] << (64 - sh));
        }
        return g.at(p);
    }
};

// Extend h while text[i+h] == text[j+h] and h < lim, one word of characters
// per step, for at most `steps` steps.  Returns true when the lcp is final.
template <class TI, class P>
__device__ __forceinline__ bool extend_short(const TI &ti, const Sym &g, ix_t<P> i, ix_t<P> j,
                                             P &h, P lim, int steps) {
    using IX = ix_t<P>;
    const int per = g.per();
    for (int it = 0; it < steps; ++it) {
        if (h >= lim) { h = lim; return true; }
        const uint64_t x = ti.at(IX(i + IX(h))) ^ g.at(IX(j + IX(h)));
        if (x) {
            const IX nh = IX(h) + IX(__builtin_ctzll(x) >> g.lg);  // below 2^32: h < 2^31
            h = nh < IX(lim) ? P(nh) : lim;
            return true;
        }
        const IX nh = IX(h) + IX(per);
        h = nh < IX(lim) ? P(nh) : lim;
    }
    if (h >= lim) { h = lim; return true; }
    return false;
}

// Wave-cooperative extension for lanes whose compare is still running: the
// lanes that want it are served one after another, and for each the whole
// wave compares two words of both suffixes per lane and round (both sides are
// contiguous, so the loads coalesce).  Must be reached by every lane of the
// wave.
template <class P>
__device__ __forceinline__ void extend_wave(bool want, const Sym &g, ix_t<P> i, ix_t<P> j,
                                            P &h, P lim) {
    using IX = ix_t<P>;  // lh + one round stays below 2^32 (lh < lim < 2^31)
    const int per = g.per();
    uint64_t mask = __ballot(want);
    while (mask) {
        const int leader = __ffsll((long long)mask) - 1;
        const IX li = __shfl(i, leader);
        const IX lj = __shfl(j, leader);
        const IX llim = IX(__shfl(lim, leader));
        IX lh = IX(__shfl(h, leader));
        while (lh < llim) {
            const IX off = lh + IX(lane()) * 2 * per;
            int mm = 2 * per;  // first mismatching character in this lane's run
            const bool inr = off < llim;
            if (inr) {
                const uint64_t x0 = g.at(li + off) ^ g.at(lj + off);
                const uint64_t x1 = g.at(li + off + per) ^ g.at(lj + off + per);
                mm = x0 ? (__builtin_ctzll(x0) >> g.lg)
                        : (x1 ? per + (__builtin_ctzll(x1) >> g.lg) : 2 * per);
            }
            const uint64_t stop = __ballot(!inr || mm < 2 * per);
            if (stop) {
                const int fl = __ffsll((long long)stop) - 1;
                const int fm = __shfl(mm, fl);
                const IX nh = lh + IX(fl) * 2 * per + IX(fm);
                lh = nh < llim ? nh : llim;
                break;
            }
            lh += IX(WAVE) * 2 * per;
        }
        if (lane() == leader) h = P(lh < llim ? lh : llim);
        mask &= mask - 1;
    }
}

// ============================================================================
// Rank scatter (Section 3: Rank = SA^-1).  Slot g of the concatenated SA array
// belongs to segment b, rank r = g - off[b]; the suffix is i = off[b] + SA[g].
// Each suffix receives its two SA neighbours as one 8-byte store (one random
// cache line per position), and optionally its rank.
// ============================================================================

// Segment of the block's first element, found once by its first wave.
__device__ __forceinline__ int32_t block_segment(const Segs &segs, int64_t first, int32_t *s_b) {
    if (threadIdx.x < WAVE) {
        const int32_t b = segs.find_wave(first);
        if (threadIdx.x == 0) *s_b = b;
    }
    __syncthreads();
    return *s_b;
}

// The same with the segment's bounds, for the block's lanes to start from
// (SegRun::at then reloads nothing while they stay in that segment).
__device__ __forceinline__ SegRun block_segrun(const Segs &segs, int64_t first, SegRun *s_r) {
    if (threadIdx.x < WAVE) {
        const SegRun r = find_run_wave(segs, first);
        if (threadIdx.x == 0) *s_r = r;
    }
    __syncthreads();
    return *s_r;
}

// clear (optional): nclear words that block 0 sets to zero for the kernels
// that follow (saves a launch in the build path).
template <class P>
__device__ __forceinline__ void rank_scatter_body(const P *__restrict__ sa, int64_t total,
                                                  const Segs &segs, pair_t<P> *__restrict__ nbr,
                                                  P *__restrict__ rank, uint32_t *err,
                                                  uint64_t *clear, int nclear, SegRun *s_r) {
    if (clear && blockIdx.x == 0 && int(threadIdx.x) < nclear) clear[threadIdx.x] = 0;
    const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const bool in = g < total;
    // The three SA loads go out before the segment search, so that their
    // latency overlaps it.
    int64_t v = -1, up = -1, un = -1;
    if (in) {
        v = sa[g];
        if (g > 0) up = sa[g - 1];
        if (g + 1 < total) un = sa[g + 1];
    }
    // The block's first wave finds the segment of its first slot (a search
    // per wave would quadruple the probe loads).
    SegRun sr{0, 0, total};
    if (segs.off) {
        const int64_t g0 = int64_t(blockIdx.x) * blockDim.x;
        if (threadIdx.x < WAVE) {
            const SegRun r = find_run_wave(segs, g0);
            if (threadIdx.x == 0) *s_r = r;
        }
        __syncthreads();
        sr = *s_r;
    }
    if (!in) return;
    sr.at(segs, g);
    const int64_t s0 = sr.sb, s1 = sr.se;
    const int64_t len = s1 - s0;
    if (g < s0 || g >= s1) { raise_err(err, LRQ_ERR_SA); return; }
    const int64_t r = g - s0;
    if (v < 0 || v >= len) { raise_err(err, LRQ_ERR_SA); return; }
    P prev = -1, next = -1;
    if (r > 0) {  // then g > 0, and up is SA[g - 1]
        if (up >= 0 && up < len) prev = P(s0 + up); else raise_err(err, LRQ_ERR_SA);
    }
    if (r + 1 < len) {  // then g + 1 < total, and un is SA[g + 1]
        if (un >= 0 && un < len) next = P(s0 + un); else raise_err(err, LRQ_ERR_SA);
    }
    nbr[s0 + v] = mkpair<P>(prev, next);
    if (rank) rank[s0 + v] = P(r);
}

__global__ __launch_bounds__(512) void rank_scatter_kernel(const int32_t *__restrict__ sa,
                                                           int64_t total, Segs segs,
                                                           int2 *__restrict__ nbr,
                                                           int32_t *__restrict__ rank,
                                                           uint32_t *err, uint64_t *clear,
                                                           int nclear) {
    __shared__ SegRun s_r;
    rank_scatter_body<int32_t>(sa, total, segs, nbr, rank, err, clear, nclear, &s_r);
}

__global__ __launch_bounds__(512) void rank_scatter64_kernel(const int64_t *__restrict__ sa,
                                                             int64_t total, Segs segs,
                                                             longlong2 *__restrict__ nbr,
                                                             int64_t *__restrict__ rank,
                                                             uint32_t *err, uint64_t *clear,
                                                             int nclear) {
    __shared__ SegRun s_r;
    rank_scatter_body<int64_t>(sa, total, segs, nbr, rank, err, clear, nclear, &s_r);
}

// ============================================================================
// Text-order LCP.  For suffix i with preceding neighbour jp = Phi[i] and
// following neighbour jn, PLCP[i] = lcp(i, jp) = LCP[Rank[i]] and
// NLCP[i] = lcp(i, jn) = LCP[Rank[i]+1], the two terms of Lemma 1.  Kasai's
// argument gives PLCP[i+1] >= PLCP[i] - 1 and likewise for NLCP, so a lane
// that walks consecutive positions only compares the new characters.
//
// Work split: heads of level l (every stride_l-th position, coarse to fine)
// are computed exactly, each seeded from the head of level l+1 at or before it
// (PLCP[p] >= PLCP[H] - (p - H) within one string); then every lane walks a
// chunk of PLCP_CHUNK positions seeded from the level-1 head before it.
// ============================================================================

// One position: exact (PLCP, NLCP) from lower bounds (hp, hn).  xp / xn say
// that the bound is already exact, so that side compares nothing.
template <class TI, class P>
// Positions, segment bounds and neighbours are all below LRQ_MAX_TOTAL (or
// LRQ64_MAX_TOTAL) here, so they are held in P.
__device__ __forceinline__ void lcp_pair(bool act, const TI &ti, const Sym &g, P p, P sb, P se,
                                         pair_t<P> nb, P &hp, P &hn, uint32_t *err,
                                         bool xp = false, bool xn = false) {
    using IX = ix_t<P>;
    P jp = nb.x, jn = nb.y;
    P limp = 0, limn = 0;
    if (act) {
        if (jp >= 0 && (jp < sb || jp >= se || jp == p)) { raise_err(err, LRQ_ERR_PHI); jp = -1; }
        if (jn >= 0 && (jn < sb || jn >= se || jn == p)) { raise_err(err, LRQ_ERR_PHI); jn = -1; }
        if (jp < 0) hp = 0; else limp = se - (p > jp ? p : jp);
        if (jn < 0) hn = 0; else limn = se - (p > jn ? p : jn);
        if (hp > limp) hp = limp;
        if (hn > limn) hn = limn;
    } else {
        jp = jn = -1;
    }
    const IX ip = IX(p), ijp = IX(jp < 0 ? 0 : jp), ijn = IX(jn < 0 ? 0 : jn);
    const bool lp = act && jp >= 0 && !xp && !extend_short(ti, g, ip, ijp, hp, limp, 4);
    const bool ln = act && jn >= 0 && !xn && !extend_short(ti, g, ip, ijn, hn, limn, 4);
    extend_wave(lp, g, ip, ijp, hp, limp);
    extend_wave(ln, g, ip, ijn, hn, limn);
}

// Threads per head-level workgroup at least (see launch_levels).
constexpr int LEVEL_MIN_THREADS = 256;

template <class P>
struct Levels {
    int top;                                  // coarsest level
    int64_t stride[PLCP_MAX_LEVELS + 1];
    pair_t<P> *heads[PLCP_MAX_LEVELS + 1];
};

// All head levels in one launch.  Workgroup q owns the region
// [q*stride_top, (q+1)*stride_top): every head inside it is seeded only from
// heads inside it, so the levels run coarse to fine with a barrier between
// them and no grid-wide synchronisation.
template <class P>
__device__ __forceinline__ void plcp_levels_body(const uint8_t *__restrict__ text, int64_t total,
                                                 const Segs &segs,
                                                 const pair_t<P> *__restrict__ nbr,
                                                 const Levels<P> &lv, const uint64_t *packed,
                                                 int64_t pwords, const int32_t *lgp,
                                                 uint32_t *err, SegRun *s_r) {
    const int64_t R0 = int64_t(blockIdx.x) * lv.stride[lv.top];
    const int64_t R1 = imin(R0 + lv.stride[lv.top], total);
    const SegRun r0 = block_segrun(segs, R0, s_r);
    const Sym gt = make_sym(text, total, packed, pwords, lgp);
    for (int l = lv.top; l >= 1; --l) {
        const int64_t s = lv.stride[l];
        const int64_t cnt = (R1 - R0 + s - 1) / s;
        const int64_t rounds = (cnt + blockDim.x - 1) / blockDim.x;
        for (int64_t rd = 0; rd < rounds; ++rd) {
            // heads are dealt to the waves in turn (head i to wave i % W), so
            // that when a level has fewer heads than threads every wave gets
            // some, and long compares, which a wave serves one lane at a time,
            // run in several waves at once
            const int W = int(blockDim.x) / WAVE;
            const int64_t i = rd * blockDim.x + int64_t(lane()) * W + threadIdx.x / WAVE;
            const bool act = i < cnt;
            const int64_t p = act ? R0 + i * s : R0;
            P hp = 0, hn = 0;
            int64_t sb = 0, se = 0;
            pair_t<P> nb = mkpair<P>(-1, -1);
            if (act) {
                // the pair and the seeding head are loaded before the
                // segment bounds are known
                nb = nbr[p];
                const int64_t S = l < lv.top ? lv.stride[l + 1] : 1;
                const int64_t H = (p / S) * S;
                const pair_t<P> hv = l < lv.top ? lv.heads[l + 1][H / S] : mkpair<P>(0, 0);
                SegRun sr = r0;
                sr.at(segs, p);
                sb = sr.sb;
                se = sr.se;
                if (l < lv.top && H >= sb) {
                    const int64_t d = p - H;
                    hp = P(imax(0, int64_t(hv.x) - d));
                    hn = P(imax(0, int64_t(hv.y) - d));
                }
            }
            lcp_pair<Sym, P>(act, gt, gt, p, sb, se, nb, hp, hn, err);
            if (act) lv.heads[l][p / s] = mkpair<P>(hp, hn);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void plcp_levels_kernel(const uint8_t *__restrict__ text,
                                                           int64_t total, Segs segs,
                                                           const int2 *__restrict__ nbr,
                                                           Levels<int32_t> lv,
                                                           const uint64_t *packed, int64_t pwords,
                                                           const int32_t *lgp, uint32_t *err) {
    __shared__ SegRun s_r;
    plcp_levels_body<int32_t>(text, total, segs, nbr, lv, packed, pwords, lgp, err, &s_r);
}

__global__ __launch_bounds__(1024) void plcp_levels64_kernel(const uint8_t *__restrict__ text,
                                                             int64_t total, Segs segs,
                                                             const longlong2 *__restrict__ nbr,
                                                             Levels<int64_t> lv,
                                                             const uint64_t *packed,
                                                             int64_t pwords, const int32_t *lgp,
                                                             uint32_t *err) {
    __shared__ SegRun s_r;
    plcp_levels_body<int64_t>(text, total, segs, nbr, lv, packed, pwords, lgp, err, &s_r);
}

// LDS: the block's neighbour records, transposed so that step s of lane l is
// row s, column l (padded rows keep both the coalesced fill and the per-step
// reads free of bank conflicts), and the block's text plus a margin.
// A block spans PLCP_SPAN positions with PLCP_SPAN / CHUNK lanes.
constexpr int PLCP_TEXT_SYMS = PLCP_SPAN + 512;  // characters staged per block
constexpr int PLCP_TEXT_WORDS = PLCP_TEXT_SYMS / 8;  // LDS words, enough for bytes

// The chunk walk of one block: stages the block's neighbour pairs and text in
// LDS, then every lane walks its CHUNK positions.  On return (after a barrier)
// rec[s * ROW + t] holds (PLCP, NLCP) of position B0 + t * CHUNK + s.
// With COUNT, also counts along the walk the lane's positions after its first
// that the LLR filter keeps (Lemma 1's L and the keep rule of Section 4.2),
// and reports whether the lane's first position starts a string.
template <int CHUNK, bool COUNT = false, class P = int32_t>
__device__ __forceinline__ int32_t plcp_walk(const Sym &g, int64_t total,
                                             const Segs &segs, const pair_t<P> *__restrict__ nbr,
                                             const pair_t<P> *__restrict__ heads1, int64_t stride1,
                                             uint32_t *err, int64_t B0, pair_t<P> *rec,
                                             uint64_t *tx, SegRun *s_r, int32_t *kept = nullptr,
                                             bool *c0_starts = nullptr) {
    constexpr int PLCP_THREADS = PLCP_SPAN / CHUNK;
    constexpr int PLCP_ROW = PLCP_THREADS + 1;
    const int t = threadIdx.x;
    const int64_t c0 = B0 + int64_t(t) * CHUNK;
    // The level-1 head at or before the chunk is loaded with the block's
    // pairs; it seeds the chunk only if it lies in the chunk's string.
    const int64_t H = (c0 / stride1) * stride1;
    const pair_t<P> hv = heads1[c0 < total ? H / stride1 : 0];  // used only if c0 < total
    // The block's text words go out with the pairs too: words inside the
    // packed (or byte) array are loaded unconditionally, the few past its end
    // are filled in after.
    const int64_t w0 = (B0 << g.lg) >> 6;  // B0 is a multiple of 4096
    const int nw = (PLCP_TEXT_SYMS << g.lg) >> 6;
    constexpr int TXW = (PLCP_TEXT_WORDS + PLCP_THREADS - 1) / PLCP_THREADS;
    uint64_t txv[TXW];
    if (g.nwords > 0) {
#pragma unroll
        for (int q = 0; q < TXW; ++q) {
            if (q * PLCP_THREADS >= nw) break;  // the same in every lane
            const int64_t k = w0 + t + q * PLCP_THREADS;
            txv[q] = g.w[k < g.nwords ? k : g.nwords - 1];
        }
    }
    // The neighbour pairs are read once and the LCP pairs written once:
    // streaming (non-temporal) accesses leave the L2 to the packed text that
    // the neighbour-side compares read at random.
    // Eight loads at a time go out before any is stored: the index is
    // clamped instead of branched on, since a load inside a branch of its
    // own is waited for there, one round trip per pair.
    constexpr int BATCH = CHUNK < 8 ? CHUNK : 8;
#pragma unroll
    for (int e0 = 0; e0 < CHUNK; e0 += BATCH) {
        pair_t<P> v[BATCH];
#pragma unroll
        for (int e = 0; e < BATCH; ++e) {
            const int64_t p = B0 + (e0 + e) * PLCP_THREADS + t;
            v[e] = load_stream(nbr + (p < total ? p : total - 1));
        }
#pragma unroll
        for (int e = 0; e < BATCH; ++e) {
            const int idx = (e0 + e) * PLCP_THREADS + t;
            rec[(idx % CHUNK) * PLCP_ROW + idx / CHUNK] =
                B0 + idx < total ? v[e] : mkpair<P>(-1, -1);
        }
    }
#pragma unroll
    for (int q = 0; q < TXW; ++q) {
        const int w = t + q * PLCP_THREADS;
        const int64_t k = w0 + w;
        if (w < nw) tx[w] = k < g.nwords ? txv[q] : g.word(k);
    }
    SegRun sr = block_segrun(segs, B0, s_r);  // includes the barrier
    const int32_t bblk = sr.b;

    const StagedSym st{g, tx, B0, PLCP_TEXT_SYMS};
    P hp = 0, hn = 0;
    int32_t b = bblk;
    int64_t sb = 0, se = 0;
    if (c0 < total) {
        sr.at(segs, c0);
        b = sr.b;
        sb = sr.sb;
        se = sr.se;
        if (H >= sb) {
            const int64_t d = c0 - H;
            hp = P(imax(0, int64_t(hv.x) - d));
            hn = P(imax(0, int64_t(hv.y) - d));
        }
    }
    // Kasai's step made exact: if lcp(p-1, j) = h >= 1 then lcp(p, j+1) = h - 1,
    // so when p's neighbour is the successor of the previous position's
    // neighbour the carried bound is the value and no text is read.
    int64_t pjp = -1, pjn = -1;  // previous position's neighbours, when its lcp >= 1
    P prevL = 0;
    int32_t cnt = 0;
    if (COUNT) *c0_starts = c0 < total && c0 == sb;
    for (int s = 0; s < CHUNK; ++s) {
        const int64_t p = c0 + s;
        const bool act = p < total;
        if (act && p >= se) {  // a new string starts inside the chunk
            b = segs.advance(b, p);
            sb = segs.begin(b);
            se = segs.end(b);
            hp = hn = 0;
            pjp = pjn = -1;
            prevL = 0;
        }
        const pair_t<P> nb = rec[s * PLCP_ROW + t];
        const bool xp = pjp >= 0 && nb.x == pjp + 1;
        const bool xn = pjn >= 0 && nb.y == pjn + 1;
        lcp_pair<StagedSym, P>(act, st, g, p, sb, se, nb, hp, hn, err, xp, xn);
        if (act) rec[s * PLCP_ROW + t] = mkpair<P>(hp, hn);
        if (COUNT) {
            const P L = hp > hn ? hp : hn;
            if (s > 0 && act && L > 0 && L >= prevL) ++cnt;
            prevL = L;
        }
        pjp = act && hp >= 1 ? nb.x : -1;
        pjn = act && hn >= 1 ? nb.y : -1;
        hp = hp > 0 ? hp - 1 : 0;
        hn = hn > 0 ? hn - 1 : 0;
    }
    if (COUNT) *kept = cnt;
    __syncthreads();
    return bblk;
}

// Lw (optional): write Lemma 1's L = max(PLCP, NLCP) of every position there
// instead of the (PLCP, NLCP) pairs over pn (the build path, whose filter
// needs only L).
template <int CHUNK>
__device__ __forceinline__ void plcp_chunks_body(
    const uint8_t *__restrict__ text, int64_t total, const Segs &segs, int2 *__restrict__ pn,
    const int2 *__restrict__ heads1, int64_t stride1, const uint64_t *packed, int64_t pwords,
    const int32_t *lgp, uint32_t *err, int4 *__restrict__ keepsum, int32_t *__restrict__ Lw) {
    constexpr int PLCP_THREADS = PLCP_SPAN / CHUNK;
    constexpr int PLCP_ROW = PLCP_THREADS + 1;
    __shared__ int2 rec[CHUNK * PLCP_ROW];
    __shared__ uint64_t tx[PLCP_TEXT_WORDS];
    __shared__ SegRun s_r;
    __shared__ int32_t s_cnt[PLCP_THREADS / WAVE];
    const int t = threadIdx.x;
    const int64_t B0 = int64_t(blockIdx.x) * PLCP_SPAN;
    const Sym g = make_sym(text, total, packed, pwords, lgp);
    // In place: the block reads only its own neighbour pairs (staged first),
    // then overwrites them with its LCP pairs.
    if (keepsum) {
        // The block's share of the LLR filter's count for every position but
        // the first, whose keep rule needs L of the previous block's last
        // position: the block records that first L, whether the block starts
        // a string, and its own last L, and the scan over blocks decides the
        // first positions.
        int32_t cnt;
        bool c0_starts;
        const int32_t bblk = plcp_walk<CHUNK, true>(g, total, segs, pn, heads1, stride1, err, B0,
                                                    rec, tx, &s_r, &cnt, &c0_starts);
        if (t > 0 && !c0_starts && B0 + int64_t(t) * CHUNK < total) {
            const int2 u = rec[(CHUNK - 1) * PLCP_ROW + t - 1];
            const int2 v = rec[t];
            const int32_t Lu = u.x > u.y ? u.x : u.y, Lv = v.x > v.y ? v.x : v.y;
            if (Lv > 0 && Lv >= Lu) ++cnt;
        } else if (t > 0 && c0_starts) {
            const int2 v = rec[t];
            if (v.x > 0 || v.y > 0) ++cnt;
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
        if (lane() == 0) s_cnt[t / WAVE] = cnt;
        __syncthreads();
        if (t == 0) {
            int32_t sum = 0;
            for (int q = 0; q < PLCP_THREADS / WAVE; ++q) sum += s_cnt[q];
            const int64_t last = (total - B0 < PLCP_SPAN ? total - B0 : PLCP_SPAN) - 1;
            const int2 vf = rec[0];
            const int2 vl = rec[(last % CHUNK) * PLCP_ROW + last / CHUNK];
            keepsum[blockIdx.x] = make_int4(sum, vf.x > vf.y ? vf.x : vf.y,
                                            B0 == segs.begin(bblk) ? 1 : 0,
                                            vl.x > vl.y ? vl.x : vl.y);
        }
    } else {
        plcp_walk<CHUNK>(g, total, segs, pn, heads1, stride1, err, B0, rec, tx, &s_r);
    }
    if (Lw) {
#pragma unroll
        for (int e = 0; e < CHUNK; ++e) {
            const int idx = e * PLCP_THREADS + t;
            const int64_t p = B0 + idx;
            const int2 v = rec[(idx % CHUNK) * PLCP_ROW + idx / CHUNK];
            if (p < total) __builtin_nontemporal_store(v.x > v.y ? v.x : v.y, Lw + p);
        }
        return;
    }
#pragma unroll
    for (int e = 0; e < CHUNK; ++e) {
        const int idx = e * PLCP_THREADS + t;
        const int64_t p = B0 + idx;
        if (p < total) store_stream(pn + p, rec[(idx % CHUNK) * PLCP_ROW + idx / CHUNK]);
    }
}

// The walk writing (PLCP, NLCP) over the neighbour pairs (lrq_plcp).
template <int CHUNK>
__global__ __launch_bounds__(PLCP_SPAN / CHUNK) void plcp_chunks_kernel(
    const uint8_t *__restrict__ text, int64_t total, Segs segs, int2 *__restrict__ pn,
    const int2 *__restrict__ heads1, int64_t stride1, const uint64_t *packed, int64_t pwords,
    const int32_t *lgp, uint32_t *err, int4 *__restrict__ keepsum) {
    plcp_chunks_body<CHUNK>(text, total, segs, pn, heads1, stride1, packed, pwords, lgp, err,
                            keepsum, nullptr);
}

// The walk writing L alone (the build path; its filter needs only L).
template <int CHUNK>
__global__ __launch_bounds__(PLCP_SPAN / CHUNK) void plcp_chunks_l_kernel(
    const uint8_t *__restrict__ text, int64_t total, Segs segs, int2 *__restrict__ pn,
    const int2 *__restrict__ heads1, int64_t stride1, const uint64_t *packed, int64_t pwords,
    const int32_t *lgp, uint32_t *err, int4 *__restrict__ keepsum, int32_t *__restrict__ Lw) {
    plcp_chunks_body<CHUNK>(text, total, segs, pn, heads1, stride1, packed, pwords, lgp, err,
                            keepsum, Lw);
}

// The chunk walk with 64-bit positions and lengths (no keep summaries: the
// 64-bit build runs the filter with its own look-back).
template <int CHUNK>
__global__ __launch_bounds__(PLCP_SPAN / CHUNK) void plcp_chunks64_kernel(
    const uint8_t *__restrict__ text, int64_t total, Segs segs, longlong2 *__restrict__ pn,
    const longlong2 *__restrict__ heads1, int64_t stride1, const uint64_t *packed,
    int64_t pwords, const int32_t *lgp, uint32_t *err) {
    constexpr int PLCP_THREADS = PLCP_SPAN / CHUNK;
    constexpr int PLCP_ROW = PLCP_THREADS + 1;
    __shared__ longlong2 rec[CHUNK * PLCP_ROW];
    __shared__ uint64_t tx[PLCP_TEXT_WORDS];
    __shared__ SegRun s_r;
    const int t = threadIdx.x;
    const int64_t B0 = int64_t(blockIdx.x) * PLCP_SPAN;
    const Sym g = make_sym(text, total, packed, pwords, lgp);
    plcp_walk<CHUNK, false, int64_t>(g, total, segs, pn, heads1, stride1, err, B0, rec, tx, &s_r);
#pragma unroll
    for (int e = 0; e < CHUNK; ++e) {
        const int idx = e * PLCP_THREADS + t;
        const int64_t p = B0 + idx;
        if (p < total) store_stream(pn + p, rec[(idx % CHUNK) * PLCP_ROW + idx / CHUNK]);
    }
}

// ============================================================================
// LLR filter: Lemma 1's L_i = max(PLCP[i], NLCP[i]), the keep rule of
// Section 4.2 (L_i > 0 and L_i >= L_{i-1}), and the compaction of Section 5.2
// (flag, prefix sum, scatter) fused into one pass with a decoupled look-back
// across tiles.  Lane l of a wave handles positions 2(64k + l) + {0,1} of the
// wave's span in load k, so every 16-byte load is contiguous across the wave
// and the in-order rank of a kept position is a popcount of two ballots.
// Each wave span is one LRQ_BLOCK of positions; the wave also records how many
// compact entries start before its span (the block table).
// ============================================================================

constexpr uint64_t DESC_AGG = 1ull << 62;
constexpr uint64_t DESC_PFX = 2ull << 62;
constexpr uint64_t DESC_VAL = (1ull << 62) - 1;
constexpr uint32_t SPIN_LIMIT = 1u << 22;

__device__ __forceinline__ uint64_t desc_load(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void desc_store(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t *s_tmp, int64_t &total) {
    // s_tmp: blockDim.x / WAVE entries
    const int l = lane(), w = threadIdx.x / WAVE;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const int64_t y = __shfl_up(x, o);
        if (l >= o) x += y;
    }
    if (l == WAVE - 1) s_tmp[w] = x;
    __syncthreads();
    int64_t pre = 0;
    total = 0;
    for (int q = 0; q < int(blockDim.x / WAVE); ++q) {
        if (q < w) pre += s_tmp[q];
        total += s_tmp[q];
    }
    __syncthreads();
    return pre + x - v;
}

__device__ __forceinline__ int64_t wave_sum(int64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Called by every lane of one wave.  Publishes the tile aggregate, walks back
// over predecessors (64 at a time) until one with an inclusive prefix, and
// publishes the tile's inclusive prefix.  Tiles are claimed in ticket order by
// running blocks, so every awaited predecessor is being processed; the wait is
// still bounded (LRQ_ERR_TIMEOUT) so that no wave can spin forever.
// The look-back in two calls, so that a block can do other work between
// publishing its aggregate and waiting for its predecessors.
__device__ __forceinline__ void look_back_publish(uint64_t *desc, int64_t tile, int64_t agg) {
    if (lane() == 0) desc_store(&desc[tile], (tile == 0 ? DESC_PFX : DESC_AGG) | uint64_t(agg));
}

__device__ int64_t look_back_resolve(uint64_t *desc, int64_t tile, int64_t agg, uint32_t *err) {
    const int l = lane();
    if (tile == 0) return 0;
    int64_t excl = 0;
    int64_t t = tile - 1;
    uint32_t spins = 0;
    while (true) {
        const int64_t idx = t - l;
        uint64_t d = idx >= 0 ? desc_load(&desc[idx]) : DESC_PFX;
        while (__ballot((d >> 62) == 0)) {
            if (++spins > SPIN_LIMIT) {
                if (l == 0) raise_err(err, LRQ_ERR_TIMEOUT);
                if ((d >> 62) == 0) d = DESC_PFX;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            if ((d >> 62) == 0) d = desc_load(&desc[idx]);
        }
        const uint64_t pm = __ballot((d >> 62) == 2);
        const int64_t val = int64_t(d & DESC_VAL);
        if (pm) {
            const int fl = __ffsll((long long)pm) - 1;
            excl += wave_sum(l <= fl ? val : 0);
            break;
        }
        excl += wave_sum(val);
        t -= WAVE;
    }
    if (l == 0) desc_store(&desc[tile], DESC_PFX | uint64_t(excl + agg));
    return excl;
}

__device__ __forceinline__ int64_t look_back(uint64_t *desc, int64_t tile, int64_t agg,
                                             uint32_t *err) {
    look_back_publish(desc, tile, agg);
    return look_back_resolve(desc, tile, agg, err);
}

// Exclusive bases in the compact array of every PLCP_SPAN block, from the
// blocks' keep summaries (count of kept positions after the first; L of the
// first position; whether the block starts a string; L of the last
// position).  One block; each round takes BASES_THREADS * BASES_ITEMS
// consecutive blocks, BASES_ITEMS per thread, all loads issued together and
// one round ahead.
// Also writes the compact array's length and the block table's closing entry.
constexpr int BASES_THREADS = 1024;
constexpr int BASES_ITEMS = 4;

__global__ __launch_bounds__(BASES_THREADS) void llr_bases_kernel(
    const int4 *__restrict__ keepsum, int64_t nb, int64_t *__restrict__ base, int64_t total,
    int64_t *__restrict__ llrc_count, int64_t *__restrict__ blocks) {
    __shared__ int64_t s_tmp[BASES_THREADS / WAVE];
    constexpr int64_t ROUND = int64_t(BASES_THREADS) * BASES_ITEMS;
    int64_t carry = 0;
    // the next round's summaries are loaded while this round is scanned
    int4 nxt[BASES_ITEMS];
    int32_t nxt_last;
    auto load = [&](int64_t r0) {
        const int64_t j0 = r0 + int64_t(threadIdx.x) * BASES_ITEMS;
#pragma unroll
        for (int i = 0; i < BASES_ITEMS; ++i)
            nxt[i] = j0 + i < nb ? keepsum[j0 + i] : make_int4(0, 0, 0, 0);
        nxt_last = j0 > 0 && j0 < nb ? keepsum[j0 - 1].w : 0;
    };
    load(0);
    for (int64_t r0 = 0; r0 < nb; r0 += ROUND) {
        const int64_t j0 = r0 + int64_t(threadIdx.x) * BASES_ITEMS;
        int4 cur[BASES_ITEMS];
#pragma unroll
        for (int i = 0; i < BASES_ITEMS; ++i) cur[i] = nxt[i];
        int32_t prev_last = nxt_last;
        if (r0 + ROUND < nb) load(r0 + ROUND);
        int64_t c[BASES_ITEMS];
        int64_t sum = 0;
#pragma unroll
        for (int i = 0; i < BASES_ITEMS; ++i) {
            const int64_t j = j0 + i;
            const bool first =
                cur[i].y > 0 && (cur[i].z != 0 || j == 0 || cur[i].y >= prev_last);
            c[i] = j < nb ? int64_t(cur[i].x) + (first ? 1 : 0) : 0;
            sum += c[i];
            prev_last = cur[i].w;
        }
        int64_t all;
        int64_t run = carry + block_exclusive_scan(sum, s_tmp, all);
#pragma unroll
        for (int i = 0; i < BASES_ITEMS; ++i) {
            if (j0 + i < nb) base[j0 + i] = run;
            run += c[i];
        }
        carry += all;
    }
    if (threadIdx.x == 0) {
        *llrc_count = carry;
        blocks[(total + LRQ_BLOCK - 1) / LRQ_BLOCK] = carry;
    }
}

// tile_base: when given, the exclusive base of every PLCP_SPAN block
// (llr_bases_kernel), and tiles are taken in launch order with no look-back;
// otherwise tiles are claimed by ticket and chained by the look-back.
// FROM_L: the input holds Lemma 1's lengths L (P[total], e.g. written by the
// LCP walk of lrq_index_build) instead of (PLCP, NLCP) pairs; L is then not
// written again.
template <int WAVES, class P, bool FROM_L = false>
__device__ __forceinline__ void llr_filter_body(
    const pair_t<P> *__restrict__ pn, int64_t total, const Segs &segs,
    pair_t<P> *__restrict__ llrc, int64_t *__restrict__ llrc_count, int64_t *__restrict__ blocks,
    P *__restrict__ Lout, uint64_t *desc, uint32_t *ticket, uint32_t *err, int64_t ntiles,
    const int64_t *__restrict__ tile_base, int64_t *s_tile, int64_t *s_wave, int64_t *s_base) {
    using E = pair_t<P>;
    constexpr int LLR_THREADS = WAVES * 64;
    constexpr int LLR_TILE = WAVES * LLR_WAVE_SPAN;
    static_assert(LLR_TILE % PLCP_SPAN == 0, "a filter tile covers whole PLCP blocks");
    int64_t tile = blockIdx.x;
    if (!tile_base) {
        if (threadIdx.x == 0) *s_tile = atomicAdd(ticket, 1u);
        __syncthreads();
        tile = *s_tile;
    }
    const int64_t given_base = tile_base ? tile_base[tile * (LLR_TILE / PLCP_SPAN)] : 0;
    const int w = threadIdx.x / WAVE, l = lane();
    const int64_t wb = tile * LLR_TILE + int64_t(w) * LLR_WAVE_SPAN;

    // Segment of this lane's first position (found once per wave), advanced
    // as positions grow.
    SegRun sr{0, 0, total};
    if (segs.off) {
        sr = find_run_wave(segs, wb);
        sr.at(segs, wb + 2 * l);
    }

    // All loads of the wave's span are issued before any is used, so a wave
    // waits for memory once rather than once per load.  Lane l holds the
    // pairs of positions 2(64k + l) and 2(64k + l) + 1: one 16-byte load for
    // 32-bit pairs, two for 64-bit ones.
    // With FROM_L, A[k] holds (L[p0], L[p0 + 1]) (one load of a pair-sized
    // word) and B is unused.
    const P *Lin = reinterpret_cast<const P *>(pn);
    E A[LLR_LOADS], B[LLR_LOADS];
    const E Z = mkpair<P>(0, 0);
    if (wb + LLR_WAVE_SPAN <= total) {  // the whole span is in range
#pragma unroll
        for (int k = 0; k < LLR_LOADS; ++k) {
            const int64_t p0 = wb + 2 * (int64_t(k) * WAVE + l);
            if constexpr (FROM_L) {
                A[k] = pn[p0 >> 1];
            } else if constexpr (sizeof(P) == 4) {
                const int4 q = reinterpret_cast<const int4 *>(pn)[p0 >> 1];
                A[k] = make_int2(q.x, q.y);
                B[k] = make_int2(q.z, q.w);
            } else {
                A[k] = pn[p0];
                B[k] = pn[p0 + 1];
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < LLR_LOADS; ++k) {
            const int64_t p0 = wb + 2 * (int64_t(k) * WAVE + l);
            if constexpr (FROM_L) {
                A[k] = mkpair<P>(p0 < total ? Lin[p0] : P(0), p0 + 1 < total ? Lin[p0 + 1] : P(0));
            } else {
                A[k] = p0 < total ? pn[p0] : Z;
                B[k] = p0 + 1 < total ? pn[p0 + 1] : Z;
            }
        }
    }
    // L of the position before the wave's span, straight from the input.
    P carry = 0;
    if (wb > 0 && wb - 1 < total) {
        if constexpr (FROM_L) {
            carry = Lin[wb - 1];
        } else {
            const E q = pn[wb - 1];
            carry = q.x > q.y ? q.x : q.y;
        }
    }
    P L0[LLR_LOADS], L1[LLR_LOADS];
    uint64_t m0[LLR_LOADS], m1[LLR_LOADS];
    int64_t wave_total = 0;
#pragma unroll
    for (int k = 0; k < LLR_LOADS; ++k) {
        const int64_t p0 = wb + 2 * (int64_t(k) * WAVE + l);
        P a0, a1;
        if constexpr (FROM_L) {
            a0 = A[k].x;
            a1 = A[k].y;
        } else {
            a0 = A[k].x > A[k].y ? A[k].x : A[k].y;
            a1 = B[k].x > B[k].y ? B[k].x : B[k].y;
        }
        const P up = __shfl_up(a1, 1);
        P prev0 = l == 0 ? carry : up;
        P prev1 = a0;
        carry = __shfl(a1, WAVE - 1);
        // L_{-1} = 0 at the first position of every string.
        if (p0 < total) {
            sr.at(segs, p0);
            if (p0 == sr.sb) prev0 = 0;
        }
        if (p0 + 1 < total) {
            sr.at(segs, p0 + 1);
            if (p0 + 1 == sr.sb) prev1 = 0;
        }
        const bool k0 = p0 < total && a0 > 0 && a0 >= prev0;
        const bool k1 = p0 + 1 < total && a1 > 0 && a1 >= prev1;
        L0[k] = a0;
        L1[k] = a1;
        m0[k] = __ballot(k0);
        m1[k] = __ballot(k1);
        wave_total += __popcll(m0[k]) + __popcll(m1[k]);
        if (!FROM_L && Lout) {
            if (p0 + 1 < total) {
                reinterpret_cast<E *>(Lout)[p0 >> 1] = mkpair<P>(a0, a1);
            } else if (p0 < total) {
                Lout[p0] = a0;
            }
        }
    }
    if (l == 0) s_wave[w] = wave_total;
    __syncthreads();
    if (!tile_base && w == 0) {
        int64_t agg = 0;
        for (int q = 0; q < LLR_THREADS / WAVE; ++q) agg += s_wave[q];
        const int64_t excl = look_back(desc, tile, agg, err);
        if (l == 0) {
            *s_base = excl;
            if (tile == ntiles - 1) {
                *llrc_count = excl + agg;
                blocks[(total + LRQ_BLOCK - 1) / LRQ_BLOCK] = excl + agg;
            }
        }
    }
    __syncthreads();
    int64_t base = tile_base ? given_base : *s_base;
    for (int q = 0; q < w; ++q) base += s_wave[q];
    if (l == 0 && wb < total) blocks[wb / LRQ_BLOCK] = base;
    const uint64_t lt = (1ull << l) - 1;
#pragma unroll
    for (int k = 0; k < LLR_LOADS; ++k) {
        const int64_t p0 = wb + 2 * (int64_t(k) * WAVE + l);
        const bool k0 = (m0[k] >> l) & 1, k1 = (m1[k] >> l) & 1;
        const int64_t r = base + __popcll(m0[k] & lt) + __popcll(m1[k] & lt);
        if (k0) llrc[r] = mkpair<P>(P(p0), L0[k]);
        if (k1) llrc[r + (k0 ? 1 : 0)] = mkpair<P>(P(p0 + 1), L1[k]);
        base += __popcll(m0[k]) + __popcll(m1[k]);
    }
}

#define LLR_FILTER_PARAMS(P)                                                                    \
    const pair_t<P> *__restrict__ pn, int64_t total, Segs segs, pair_t<P> *__restrict__ llrc,   \
        int64_t *__restrict__ llrc_count, int64_t *__restrict__ blocks, P *__restrict__ Lout,   \
        uint64_t *desc, uint32_t *ticket, uint32_t *err, int64_t ntiles,                        \
        const int64_t *__restrict__ tile_base
#define LLR_FILTER_BODY(P)                                                                      \
    __shared__ int64_t s_tile, s_base;                                                          \
    __shared__ int64_t s_wave[WAVES];                                                           \
    llr_filter_body<WAVES, P>(pn, total, segs, llrc, llrc_count, blocks, Lout, desc, ticket,     \
                              err, ntiles, tile_base, &s_tile, s_wave, &s_base)

template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void llr_filter_kernel(LLR_FILTER_PARAMS(int32_t)) {
    LLR_FILTER_BODY(int32_t);
}
template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void llr_filter64_kernel(LLR_FILTER_PARAMS(int64_t)) {
    LLR_FILTER_BODY(int64_t);
}
// The build path's filter: L from the LCP walk instead of (PLCP, NLCP) pairs
// (pn then points at L, read two values per lane and load).
template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void llr_filter_l_kernel(LLR_FILTER_PARAMS(int32_t)) {
    __shared__ int64_t s_tile, s_base;
    __shared__ int64_t s_wave[WAVES];
    llr_filter_body<WAVES, int32_t, true>(pn, total, segs, llrc, llrc_count, blocks, Lout, desc,
                                          ticket, err, ntiles, tile_base, &s_tile, s_wave,
                                          &s_base);
}
#undef LLR_FILTER_PARAMS
#undef LLR_FILTER_BODY

// Text-order LCP and the LLR filter in one kernel (the build path): after the
// chunk walk the block holds (PLCP, NLCP) of its PLCP_SPAN positions in LDS,
// so Lemma 1, the keep rule and the compaction run there, with a look-back
// across blocks claimed in ticket order.  The neighbour pairs are read only,
// so the L of the position before the block is recomputed (one seeded lcp
// pair) rather than taken from a neighbour block's output.
template <int CHUNK>
__global__ __launch_bounds__(PLCP_SPAN / CHUNK) void plcp_llr_kernel(
    const uint8_t *__restrict__ text, int64_t total, Segs segs, const int2 *__restrict__ nbr,
    const int2 *__restrict__ heads1, int64_t stride1, int2 *__restrict__ llrc,
    int64_t *__restrict__ llrc_count, int64_t *__restrict__ blocks, int32_t *__restrict__ Lout,
    uint64_t *desc, uint32_t *ticket, const uint64_t *packed, int64_t pwords, const int32_t *lgp,
    uint32_t *err, int64_t ntiles) {
    constexpr int PLCP_THREADS = PLCP_SPAN / CHUNK;
    constexpr int PLCP_ROW = PLCP_THREADS + 1;
    __shared__ int2 rec[CHUNK * PLCP_ROW];
    __shared__ uint64_t tx[PLCP_TEXT_WORDS];
    __shared__ int64_t s_tmp[PLCP_THREADS / WAVE];
    __shared__ int64_t s_tile, s_base;
    __shared__ SegRun s_r;
    __shared__ int32_t s_prevL;
    const int t = threadIdx.x;
    if (t == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t B0 = tile * PLCP_SPAN;
    const Sym g = make_sym(text, total, packed, pwords, lgp);
    const int32_t bblk = plcp_walk<CHUNK>(g, total, segs, nbr, heads1, stride1, err, B0, rec,
                                          tx, &s_r);
    // L of position B0 - 1 (0 if B0 starts a string), computed by wave 0.
    if (t < WAVE) {
        const int64_t p = B0 - 1;
        bool act = t == 0 && B0 > 0 && p < total;
        int64_t sb = 0, se = 0;
        int2 nb = make_int2(-1, -1);
        int32_t hp = 0, hn = 0;
        if (act) {
            const int32_t b = segs.find(p);
            sb = segs.begin(b);
            se = segs.end(b);
            act = B0 < se;                  // B0 is in the same string as B0 - 1
            nb = nbr[p];
            const int64_t H = (p / stride1) * stride1;
            if (H >= sb) {
                const int2 hv = heads1[H / stride1];
                const int64_t d = p - H;
                hp = int32_t(imax(0, int64_t(hv.x) - d));
                hn = int32_t(imax(0, int64_t(hv.y) - d));
            }
        }
        lcp_pair<Sym, int32_t>(act, g, g, p, sb, se, nb, hp, hn, err);
        if (t == 0) s_prevL = act ? (hp > hn ? hp : hn) : 0;
    }
    __syncthreads();
    // Lemma 1 and the keep rule along the lane's chunk
    const int64_t c0 = B0 + int64_t(t) * CHUNK;
    int32_t prevL = 0;
    if (t == 0) {
        prevL = s_prevL;
    } else {
        const int2 v = rec[(CHUNK - 1) * PLCP_ROW + t - 1];
        prevL = v.x > v.y ? v.x : v.y;
    }
    SegRun sr;
    sr.init(segs, bblk, c0 < total ? c0 : B0);
    uint32_t keep = 0;
    int64_t cnt = 0;
#pragma unroll
    for (int s = 0; s < CHUNK; ++s) {
        const int64_t p = c0 + s;
        if (p >= total) break;
        sr.at(segs, p);
        if (p == sr.sb) prevL = 0;
        const int2 v = rec[s * PLCP_ROW + t];
        const int32_t L = v.x > v.y ? v.x : v.y;
        if (L > 0 && L >= prevL) {
            keep |= 1u << s;
            ++cnt;
        }
        prevL = L;
    }
    __syncthreads();  // every lane has read its left neighbour's last pair
#pragma unroll
    for (int s = 0; s < CHUNK; ++s) {
        const int2 v = rec[s * PLCP_ROW + t];
        rec[s * PLCP_ROW + t].x = v.x > v.y ? v.x : v.y;
    }
    int64_t agg;
    const int64_t ex = block_exclusive_scan(cnt, s_tmp, agg);
    if (t < WAVE) {
        const int64_t excl = look_back(desc, tile, agg, err);
        if (t == 0) {
            s_base = excl;
            if (tile == ntiles - 1) {
                *llrc_count = excl + agg;
                blocks[(total + LRQ_BLOCK - 1) / LRQ_BLOCK] = excl + agg;
            }
        }
    }
    __syncthreads();
    int64_t w = s_base + ex;
    if (c0 < total && (int64_t(t) * CHUNK) % LRQ_BLOCK == 0) blocks[c0 / LRQ_BLOCK] = w;
#pragma unroll
    for (int s = 0; s < CHUNK; ++s)
        if ((keep >> s) & 1) llrc[w++] = make_int2(int32_t(c0 + s), rec[s * PLCP_ROW + t].x);
    if (Lout) {
#pragma unroll
        for (int e = 0; e < CHUNK; ++e) {
            const int idx = e * PLCP_THREADS + t;
            const int64_t p = B0 + idx;
            if (p < total) Lout[p] = rec[(idx % CHUNK) * PLCP_ROW + idx / CHUNK].x;
        }
    }
}

// The paper's own GPU input: Rank and SA-order LCP (LCP[0] = LCP[n] = 0).
// Gathers (LCP[Rank[i]], LCP[Rank[i]+1]) into text order; the filter above
// then runs unchanged.
__global__ __launch_bounds__(256) void gather_rank_lcp_kernel(const int32_t *__restrict__ rank,
                                                              const int32_t *__restrict__ lcp,
                                                              int64_t n, int2 *__restrict__ pn,
                                                              uint32_t *err) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t r = rank[i];
    if (r < 0 || r >= n) {
        raise_err(err, LRQ_ERR_SA);
        pn[i] = make_int2(0, 0);
        return;
    }
    pn[i] = make_int2(lcp[r], lcp[r + 1]);
}

// ============================================================================
// Covering-window scan (Sections 4.2 and 5.2).  The compact entries covering k
// are the contiguous index range [a(k), z(k)): a(k) counts the entries that end
// before k, z(k) the entries that start at or before k (starts and ends of the
// compact array both increase strictly).  A block owns LR_TILE positions:
//   1. the block table gives the entries that start inside the tile, and a
//      64-wide backward ballot the ones that start before it and still cover
//      its first position; that entry range is staged in LDS;
//   2. every staged entry sets the bit of its start and the bit of its end in
//      two tile bitmaps (starts are distinct, and so are ends);
//   3. with per-word prefix popcounts, a(k) and z(k) are two popcounts each,
//      so every position is independent: lane t takes positions
//      K0 + 256 j + t and all stores coalesce.
// ============================================================================

template <class E>
__device__ __forceinline__ int64_t entry_end(const E &e) { return int64_t(e.x) + int64_t(e.y) - 1; }

__device__ __forceinline__ int64_t clamp64(int64_t v, int64_t lo, int64_t hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

// Number of compact entries, clamped to [0, total].
__device__ __forceinline__ int64_t entry_count(const int64_t *blocks, int64_t total) {
    return clamp64(blocks[(total + LRQ_BLOCK - 1) / LRQ_BLOCK], 0, total);
}

// Per-tile shared state.  The LDS window holds the tile's entries plus a
// margin of up to WAVE entries before them, where the entries that still
// cover the tile's first position are found.
template <int TILE, class E = int2>
struct LrShared {
    static constexpr int WORDS = TILE / 32;
    static constexpr int MARGIN = WAVE;
    static constexpr int CAP = MARGIN + TILE;  // staged entries at most
    // the fixed-width window scans read up to WIN_PAD entries past a window's
    // end (the values read there are masked out)
    static constexpr int WIN_PAD = 16;
    E win[CAP + WIN_PAD];
    uint32_t sbits[WORDS], ebits[WORDS];
    int32_t spre[WORDS], epre[WORDS];   // exclusive prefix popcounts
    int64_t lo, hi, first;
    int32_t seg, off, in_lds;
};

// The tile's entry range [lo, hi) with its start/end bitmaps.  Callers branch
// once on `staged` and pass either the LDS window (sh.win + off) or `src` to an
// inlined body, so the window loads compile to LDS reads (a runtime-selected
// pointer would be a generic one, and generic loads are slower).
template <class E>
struct LrTile {
    const E *src;  // window entries in global memory (src[0] is entry lo)
    bool staged;      // the whole window is also in LDS, from sh.win[off]
    int32_t off;
    int64_t cnt;      // entries in the window
    int64_t before;   // window entries that start before the tile
    int32_t seg;      // segment of the tile's first position
};

// Two dependent global round trips per tile: the block table, then the
// staged entries [first - margin, hi) in one batch of loads per thread.  The
// covering entries before the tile are a suffix of the margin (ends increase),
// so they are counted from LDS; only when all WAVE margin entries cover the
// tile start does a wave look further back in global memory, and the tile
// then reads its window from there.
template <int TILE, class E>
__device__ __forceinline__ LrTile<E> lr_prepare(const E *__restrict__ llrc,
                                                const int64_t *__restrict__ blocks, int64_t total,
                                                const Segs &segs, int64_t K0, int64_t K1,
                                                LrShared<TILE, E> &sh) {
    using SH = LrShared<TILE, E>;
    constexpr int LR_WORDS = SH::WORDS;
    const int t = threadIdx.x;
    if (t < WAVE) {
        // the block-table loads go out before the segment search
        int64_t m = 0, f = 0, h = 0;
        if (t == 0) {
            m = entry_count(blocks, total);
            f = blocks[K0 / LRQ_BLOCK];
            if (K1 < total) h = blocks[K1 / LRQ_BLOCK];
        }
        const int32_t seg = segs.find_wave(K0);
        if (t == 0) {
            const int64_t first = clamp64(f, 0, m);
            sh.first = first;
            // entries starting inside the tile have distinct starts, so at
            // most TILE of them (the clamp only guards against an
            // inconsistent table)
            sh.hi = clamp64(K1 >= total ? m : h, first, imin(m, first + TILE));
            sh.seg = seg;
        }
    }
    for (int w = t; w < LR_WORDS; w += LR_THREADS) sh.sbits[w] = sh.ebits[w] = 0;
    __syncthreads();
    const int64_t first = sh.first, hi = sh.hi;
    const int64_t M = imin(int64_t(SH::MARGIN), first);
    const int64_t nst = M + (hi - first);  // entries [first - M, hi), at most CAP
    auto mark = [&](const E &v) {
        const int64_t s = int64_t(v.x) - K0, f = entry_end(v) - K0;
        if (s >= 0 && s < K1 - K0) atomicOr(&sh.sbits[s >> 5], 1u << (s & 31));
        if (f >= 0 && f < K1 - K0) atomicOr(&sh.ebits[f >> 5], 1u << (f & 31));
    };
    constexpr int PER = (SH::CAP + LR_THREADS - 1) / LR_THREADS;
    if (nst > 0) {  // every load first (coalesced), then the LDS writes
        const E *base = llrc + (first - M);
        const int64_t last = nst - 1;
        E v[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int64_t q = int64_t(j) * LR_THREADS + t;
            v[j] = base[q < last ? q : last];
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int64_t q = int64_t(j) * LR_THREADS + t;
            if (q < nst) sh.win[q] = v[j];
        }
    }
    __syncthreads();
    {
        // Bit marks: thread t takes the PER consecutive staged entries from
        // PER t, ORs the bits of each bitmap word locally and issues one atomic
        // per word it touches; consecutive entries share words, so marking
        // from lanes holding consecutive entries would serialise on them.
        // Margin entries that end before K0 mark nothing.
        const int64_t q0 = int64_t(t) * PER, span = K1 - K0;
        int32_t sw = -1, ew = -1;
        uint32_t sb = 0, eb = 0;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int64_t q = q0 + u;
            if (q >= nst) break;
            const E v = sh.win[q];
            const int64_t st = int64_t(v.x) - K0, fi = entry_end(v) - K0;
            if (st >= 0 && st < span) {
                const int32_t w = int32_t(st >> 5);
                if (w != sw) {
                    if (sb) atomicOr(&sh.sbits[sw], sb);
                    sw = w;
                    sb = 0;
                }
                sb |= 1u << (st & 31);
            }
            if (fi >= 0 && fi < span) {
                const int32_t w = int32_t(fi >> 5);
                if (w != ew) {
                    if (eb) atomicOr(&sh.ebits[ew], eb);
                    ew = w;
                    eb = 0;
                }
                eb |= 1u << (fi & 31);
            }
        }
        if (sb) atomicOr(&sh.sbits[sw], sb);
        if (eb) atomicOr(&sh.ebits[ew], eb);
    }
    if (t < WAVE) {
        const int l = lane();
        const bool cov = l < M && entry_end(sh.win[M - 1 - l]) >= K0;
        const int c = __popcll(__ballot(cov));
        int64_t lo = first - c;
        if (c == SH::MARGIN) {  // the whole margin covers K0: search on in global memory
            int64_t from = lo;
            while (from > 0) {
                const int64_t e = from - 1 - l;
                const bool cv = e >= 0 && entry_end(llrc[e]) >= K0;
                const int cc = __popcll(__ballot(cv));
                from -= cc;
                if (cc < WAVE) break;
            }
            // entries [from, lo) start before the tile: only their ends can
            // fall inside it
            for (int64_t e = from + l; e < lo; e += WAVE) mark(llrc[e]);
            lo = from;
        }
        if (l == 0) {
            sh.lo = lo;
            sh.in_lds = lo >= first - M;
            sh.off = int32_t(M - (first - lo));
        }
    }
    __syncthreads();
    if (t < WAVE) {  // exclusive prefix popcounts over the words, one wave
        int32_t sacc = 0, eacc = 0;
        for (int base = 0; base < LR_WORDS; base += WAVE) {
            const int w = base + lane();
            const int32_t ps = w < LR_WORDS ? __popc(sh.sbits[w]) : 0;
            const int32_t pe = w < LR_WORDS ? __popc(sh.ebits[w]) : 0;
            int32_t xs = ps, xe = pe;
#pragma unroll
            for (int o = 1; o < WAVE; o <<= 1) {
                const int32_t ys = __shfl_up(xs, o), ye = __shfl_up(xe, o);
                if (lane() >= o) { xs += ys; xe += ye; }
            }
            if (w < LR_WORDS) {
                sh.spre[w] = sacc + xs - ps;
                sh.epre[w] = eacc + xe - pe;
            }
            sacc += __shfl(xs, WAVE - 1);
            eacc += __shfl(xe, WAVE - 1);
        }
    }
    __syncthreads();
    const int64_t lo = sh.lo;
    return LrTile<E>{llrc + lo, sh.in_lds != 0, sh.off, imax(hi - lo, 0), first - lo, sh.seg};
}

// Covering range [a, z) of tile-relative position r (window indices, below
// 2^31: a window holds at most all entries).
template <class SH, class E>
__device__ __forceinline__ void lr_range(const SH &sh, const LrTile<E> &tl, int r, int32_t &a,
                                         int32_t &z) {
    const int w = r >> 5, bit = r & 31;
    const uint32_t le = (2u << bit) - 1;  // bits 0..bit (2 << 31 wraps to 0: all bits)
    const uint32_t lt = (1u << bit) - 1;  // bits 0..bit-1
    z = int32_t(tl.before) + sh.spre[w] + __popc(sh.sbits[w] & le);
    a = sh.epre[w] + __popc(sh.ebits[w] & lt);
}

// A value every lane of the wave holds, moved to scalar registers so that the
// compiler can address stores as (scalar base + 32-bit lane offset).
__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v)));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(uint64_t(v) >> 32));
    return int64_t((uint64_t(hi) << 32) | lo);
}
// Element `i` (32-bit) of an array whose base is uniform, addressed by a
// 32-bit byte offset.
template <class T>
__device__ __forceinline__ T &elem32(T *base, uint32_t i) {
    return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + i * uint32_t(sizeof(T)));
}

// Longest entry of ws[a..z), smallest start on ties; bs = -1 if empty.
template <class E, class P>
__device__ __forceinline__ void window_max(const E *ws, int32_t a32, int32_t z32, P &bs, P &best) {
    best = 0;
    bs = -1;
    int32_t e = a32;
    for (; e + 1 < z32; e += 2) {  // two entries per step: both LDS reads issue together
        const E v0 = ws[e], v1 = ws[e + 1];
        if (v0.y > best) { best = v0.y; bs = v0.x; }
        if (v1.y > best) { best = v1.y; bs = v1.x; }
    }
    if (e < z32) {
        const E v = ws[e];
        if (v.y > best) { best = v.y; bs = v.x; }
    }
}

// The longest length in ws[a..z) (0 if empty).
template <class E>
__device__ __forceinline__ auto window_longest(const E *ws, int32_t a, int32_t z) {
    decltype(E::y) best = 0;
    int32_t e = a;
    for (; e + 1 < z; e += 2) {  // two entries per step: both LDS reads issue together
        const auto y0 = ws[e].y, y1 = ws[e + 1].y;
        best = best > y0 ? best : y0;
        best = best > y1 ? best : y1;
    }
    if (e < z) best = best > ws[e].y ? best : ws[e].y;
    return best;
}

// Records of position k in all mode: every entry of its window with the
// window's maximal length, in ascending start.
template <class E, class P>
__device__ __forceinline__ int32_t count_longest(const E *ws, int64_t a, int64_t z, P best) {
    int32_t c = 0;
    if (best > 0)
        for (int32_t e = int32_t(a); e < int32_t(z); ++e) c += ws[e].y == best;
    return c;
}

// One pass over ws[a..z): the maximal length, and the entries of that length
// as a 32-entry bit mask relative to a (all mode keeps one per position in a
// register across the tile scan; wider windows are scanned again).
template <class E, class P>
__device__ __forceinline__ void window_scan32(const E *ws, int32_t a, int32_t z, P &best,
                                              uint32_t &mask) {
    best = 0;
    mask = 0;
    uint32_t bit = 1;  // shifts out to 0 after 32 entries
    auto take = [&](P y) {
        if (y > best) {
            best = y;
            mask = bit;
        } else if (y == best) {
            mask |= bit;
        }
        bit <<= 1;
    };
    int32_t e = a;
    for (; e + 1 < z; e += 2) {  // two entries per step: both LDS reads issue together
        const P y0 = ws[e].y, y1 = ws[e + 1].y;
        take(y0);
        take(y1);
    }
    if (e < z) take(ws[e].y);
}

// The window scan in a fixed number U of steps, for a window of w <= U
// entries staged in LDS: U lengths are read from ws[a..a+U) at once
// (immediate offsets from one address), those at w or beyond count as 0, and
// the maximal length and the bit mask of the entries that have it (bit i for
// entry a + i) follow without a loop.  When the window is empty best is 0 and
// the mask is meaningless.  A wave whose windows are all short runs this
// instead of the loops above, which step to the widest window of the wave and
// pay a loop-carried branch per entry.
template <int U, class E, class P>
__device__ __forceinline__ void window_fixed(const E *ws, int32_t a, int32_t w, P &best,
                                             uint32_t &mask) {
    P y[U];
#pragma unroll
    for (int i = 0; i < U; ++i) {
        const P v = ws[a + i].y;
        y[i] = i < w ? v : P(0);
    }
    best = y[0];
#pragma unroll
    for (int i = 1; i < U; ++i) best = best > y[i] ? best : y[i];
    mask = 0;
#pragma unroll
    for (int i = U - 1; i >= 0; --i) mask = mask * 2u + uint32_t(y[i] == best);
}

// Maximal length and tie mask of a staged window (as window_scan32 for
// windows of at most 32 entries), choosing per wave between the fixed forms
// for windows of at most 4 or 8 entries and the loop.
template <class E, class P>
__device__ __forceinline__ void window_scan_staged(const E *ws, int32_t a, int32_t z, P &best,
                                                   uint32_t &mask) {
    const int32_t w = z - a;
    if (!__any(w > 8)) {
        if (!__any(w > 4)) window_fixed<4>(ws, a, w, best, mask);
        else window_fixed<8>(ws, a, w, best, mask);
    } else {
        window_scan32(ws, a, z, best, mask);
    }
}

// Longest entry of a staged window, smallest start on ties (window_max).
template <class E, class P>
__device__ __forceinline__ void window_max_staged(const E *ws, int32_t a, int32_t z, P &bs,
                                                  P &best) {
    const int32_t w = z - a;
    if (!__any(w > 8)) {
        uint32_t mask;
        if (!__any(w > 4)) window_fixed<4>(ws, a, w, best, mask);
        else window_fixed<8>(ws, a, w, best, mask);
        bs = best > 0 ? P(ws[a + __ffs(mask) - 1].x) : P(-1);
    } else {
        window_max(ws, a, z, bs, best);
    }
}

// Number of entries of maximal length in a staged window (0 if empty).
template <class E, class P>
__device__ __forceinline__ int32_t window_count_staged(const E *ws, int32_t a, int32_t z) {
    const int32_t w = z - a;
    if (!__any(w > 8)) {
        P best;
        uint32_t mask;
        if (!__any(w > 4)) window_fixed<4>(ws, a, w, best, mask);
        else window_fixed<8>(ws, a, w, best, mask);
        return best > 0 ? __popc(mask) : 0;
    }
    // two plain passes over the window (its longest length, then the
    // entries of that length) cost fewer instructions than one pass that
    // keeps a tie mask
    const P best = window_longest(ws, a, z);
    return count_longest(ws, a, z, best);
}

template <int LR_TILE, class P>
__device__ __forceinline__ void lr_leftmost_body(const pair_t<P> *__restrict__ llrc,
                                                 const int64_t *__restrict__ blocks, int64_t total,
                                                 const Segs &segs, pair_t<P> *__restrict__ out,
                                                 LrShared<LR_TILE, pair_t<P>> &sh) {
    using E = pair_t<P>;
    constexpr int LR_POS = LR_TILE / LR_THREADS;
    const int t = threadIdx.x;
    const int64_t K0 = int64_t(blockIdx.x) * LR_TILE;
    const int64_t K1 = imin(K0 + LR_TILE, total);
    const LrTile<E> tl = lr_prepare(llrc, blocks, total, segs, K0, K1, sh);
    E *const ob = out + K0;
    const int span = int(K1 - K0);
    auto body = [&](const E *ws, auto staged) {
        SegRun sr{tl.seg, 0, -1};
        // every position's window first, so that their LDS reads go out
        // together (positions past the tile's end read zeroed bitmap words)
        int32_t A[LR_POS], Z[LR_POS];
#pragma unroll
        for (int j = 0; j < LR_POS; ++j) lr_range(sh, tl, j * LR_THREADS + t, A[j], Z[j]);
#pragma unroll
        for (int j = 0; j < LR_POS; ++j) {
            const int r = j * LR_THREADS + t;
            if (r >= span) break;
            const int32_t a = A[j], z = Z[j];
            P bs, best;
            if constexpr (decltype(staged)::value) window_max_staged(ws, a, z, bs, best);
            else window_max(ws, a, z, bs, best);
            sr.at(segs, K0 + r);
            elem32(ob, r) = bs >= 0 ? mkpair<P>(P(bs - sr.sb), best) : mkpair<P>(-1, 0);
        }
    };
    if (tl.staged) body(sh.win + tl.off, std::true_type{});
    else body(tl.src, std::false_type{});
}

template <int LR_TILE>
__global__ __launch_bounds__(LR_THREADS) void lr_leftmost_kernel(
    const int2 *__restrict__ llrc, const int64_t *__restrict__ blocks, int64_t total, Segs segs,
    int2 *__restrict__ out) {
    __shared__ LrShared<LR_TILE, int2> sh;
    lr_leftmost_body<LR_TILE, int32_t>(llrc, blocks, total, segs, out, sh);
}

template <int LR_TILE>
__global__ __launch_bounds__(LR_THREADS) void lr_leftmost64_kernel(
    const longlong2 *__restrict__ llrc, const int64_t *__restrict__ blocks, int64_t total,
    Segs segs, longlong2 *__restrict__ out) {
    __shared__ LrShared<LR_TILE, longlong2> sh;
    lr_leftmost_body<LR_TILE, int64_t>(llrc, blocks, total, segs, out, sh);
}

// All-mode record count only (for sizing): one atomic add per tile.
template <int LR_TILE, class P>
__device__ __forceinline__ void lr_all_count_body(const pair_t<P> *__restrict__ llrc,
                                                  const int64_t *__restrict__ blocks,
                                                  int64_t total, const Segs &segs,
                                                  unsigned long long *grand,
                                                  LrShared<LR_TILE, pair_t<P>> &sh,
                                                  int64_t *s_tmp) {
    using E = pair_t<P>;
    constexpr int LR_POS = LR_TILE / LR_THREADS;
    const int t = threadIdx.x;
    const int64_t K0 = int64_t(blockIdx.x) * LR_TILE;
    const int64_t K1 = imin(K0 + LR_TILE, total);
    const LrTile<E> tl = lr_prepare(llrc, blocks, total, segs, K0, K1, sh);
    int64_t c = 0;
    auto body = [&](const E *ws, auto staged) {
        // every position's window first, so that their LDS reads go out
        // together (positions past the tile's end read zeroed bitmap words)
        int32_t A[LR_POS], Z[LR_POS];
#pragma unroll
        for (int j = 0; j < LR_POS; ++j) lr_range(sh, tl, j * LR_THREADS + t, A[j], Z[j]);
#pragma unroll
        for (int j = 0; j < LR_POS; ++j) {
            const int r = j * LR_THREADS + t;
            if (K0 + r >= K1) break;
            const int32_t a = A[j], z = Z[j];
            if constexpr (decltype(staged)::value) {
                c += window_count_staged<E, P>(ws, a, z);
            } else {
                // two plain passes over the window (its longest length, then
                // the entries of that length) cost fewer instructions than
                // one pass that keeps a tie mask
                const P best = window_longest(ws, a, z);
                c += count_longest(ws, a, z, best);
            }
        }
    };
    if (tl.staged) body(sh.win + tl.off, std::true_type{});
    else body(tl.src, std::false_type{});
    int64_t tot;
    block_exclusive_scan(c, s_tmp, tot);
    if (t == 0) atomicAdd(grand, (unsigned long long)tot);
}

template <int LR_TILE>
__global__ __launch_bounds__(LR_THREADS) void lr_all_count_kernel(
    const int2 *__restrict__ llrc, const int64_t *__restrict__ blocks, int64_t total, Segs segs,
    unsigned long long *grand) {
    __shared__ LrShared<LR_TILE, int2> sh;
    __shared__ int64_t s_tmp[LR_THREADS / WAVE];
    lr_all_count_body<LR_TILE, int32_t>(llrc, blocks, total, segs, grand, sh, s_tmp);
}

template <int LR_TILE>
__global__ __launch_bounds__(LR_THREADS) void lr_all_count64_kernel(
    const longlong2 *__restrict__ llrc, const int64_t *__restrict__ blocks, int64_t total,
    Segs segs, unsigned long long *grand) {
    __shared__ LrShared<LR_TILE, longlong2> sh;
    __shared__ int64_t s_tmp[LR_THREADS / WAVE];
    lr_all_count_body<LR_TILE, int64_t>(llrc, blocks, total, segs, grand, sh, s_tmp);
}

// All mode in one pass: per-position counts, their exclusive scan in position
// order inside the tile, a decoupled look-back across tiles for the tile's
// base, then offsets and records.  Records at index >= capacity are dropped
// (LRQ_ERR_CAPACITY); the grand total is published by the last tile.
template <int LR_TILE, bool LEFTMOST, class P>
__device__ __forceinline__ void lr_all_tile(
    const pair_t<P> *__restrict__ llrc, const int64_t *__restrict__ blocks, int64_t total,
    Segs segs, int64_t *__restrict__ offsets, pair_t<P> *__restrict__ recs, int64_t capacity,
    pair_t<P> *__restrict__ out, uint64_t *desc, uint32_t *ticket, int64_t *grand, uint32_t *err,
    int64_t ntiles) {
    using E = pair_t<P>;
    constexpr int LR_POS = LR_TILE / LR_THREADS;
    static_assert(LR_POS % 4 == 0, "per-thread offsets are moved as uint4");
    __shared__ LrShared<LR_TILE, E> sh;
    // record offset of every tile position relative to the tile's first
    // record: counts first, then their exclusive scan in position order
    __shared__ __align__(16) uint32_t s_off[LR_TILE];
    __shared__ int64_t s_tmp[LR_THREADS / WAVE];
    __shared__ int64_t s_tile, s_base;
    __shared__ int32_t s_fits;
    const int t = threadIdx.x;
    if (t == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const int64_t tile = uniform64(s_tile);
    const int64_t K0 = tile * LR_TILE;
    const int64_t K1 = imin(K0 + LR_TILE, total);
    const LrTile<E> tl = lr_prepare(llrc, blocks, total, segs, K0, K1, sh);

    // 1. records per position (lane t takes positions K0 + 256 j + t).  A
    //    window of at most 32 entries keeps its start and tie mask in
    //    registers for step 3; a wider one is marked by a negative start and
    //    scanned again there.
    int32_t A[LR_POS];
    uint32_t Mk[LR_POS];
    auto measure = [&](const E *ws, auto staged) {
        // every position's window first, so that their LDS reads go out
        // together (positions past the tile's end read zeroed bitmap words)
        int32_t Z[LR_POS];
#pragma unroll
        for (int j = 0; j < LR_POS; ++j) lr_range(sh, tl, j * LR_THREADS + t, A[j], Z[j]);
#pragma unroll
        for (int j = 0; j < LR_POS; ++j) {
            const int r = j * LR_THREADS + t;
            uint32_t c = 0;
            const int32_t a = A[j], z = Z[j];
            A[j] = 0;
            Mk[j] = 0;
            if (K0 + r < K1) {
                P best;
                uint32_t mask;
                if constexpr (decltype(staged)::value) window_scan_staged(ws, a, z, best, mask);
                else window_scan32(ws, a, z, best, mask);
                if (z - a <= 32) {
                    c = best > 0 ? __popc(mask) : 0;
                    A[j] = a;
                    Mk[j] = best > 0 ? mask : 0;
                } else {
                    c = uint32_t(count_longest(ws, a, z, best));
                    A[j] = -1 - a;
                }
            }
            s_off[r] = c;
        }
    };
    if (tl.staged) measure(sh.win + tl.off, std::true_type{});
    else measure(tl.src, std::false_type{});
    __syncthreads();

    // 2. exclusive scan in position order: thread t owns positions
    //    [LR_POS t, LR_POS (t+1)) of the tile
    {
        uint4 *own = reinterpret_cast<uint4 *>(s_off + LR_POS * t);
        uint32_t c[LR_POS];
        int64_t sum = 0;
#pragma unroll
        for (int q = 0; q < LR_POS / 4; ++q) {
            const uint4 v = own[q];
            c[4 * q] = v.x; c[4 * q + 1] = v.y; c[4 * q + 2] = v.z; c[4 * q + 3] = v.w;
        }
#pragma unroll
        for (int q = 0; q < LR_POS; ++q) sum += c[q];
        int64_t tile_total;
        int64_t run = block_exclusive_scan(sum, s_tmp, tile_total);
        // record offsets inside a tile are 32-bit byte offsets: 2^29 records
        // or more for a few thousand positions would be a 4 GiB output per tile
        if (tile_total >= (int64_t(1) << 29)) {
            if (t == 0) raise_err(err, LRQ_ERR_CAPACITY);
            run = 0;
        }
#pragma unroll
        for (int q = 0; q < LR_POS; ++q) {
            const uint32_t x = c[q];
            c[q] = uint32_t(run);
            run += x;
        }
#pragma unroll
        for (int q = 0; q < LR_POS / 4; ++q)
            own[q] = make_uint4(c[4 * q], c[4 * q + 1], c[4 * q + 2], c[4 * q + 3]);
        if (t < WAVE) look_back_publish(desc, tile, tile_total);
        if (LEFTMOST) {
            // the leftmost records, written while the predecessors finish
            E *const outb = out + K0;
            auto leftmost = [&](const E *ws) {
                SegRun sr{tl.seg, 0, -1};
#pragma unroll
                for (int j = 0; j < LR_POS; ++j) {
                    const int r = j * LR_THREADS + t;
                    const int64_t k = K0 + r;
                    if (k >= K1) break;
                    sr.at(segs, k);
                    const P sb = P(sr.sb);
                    E o = mkpair<P>(-1, 0);
                    if (A[j] >= 0) {
                        if (Mk[j]) {
                            const E v = ws[A[j] + __ffs(Mk[j]) - 1];
                            o = mkpair<P>(P(v.x - sb), v.y);
                        }
                    } else {
                        int32_t a, z;
                        lr_range(sh, tl, r, a, z);
                        P bs, best;
                        window_max(ws, -1 - A[j], z, bs, best);
                        if (bs >= 0) o = mkpair<P>(P(bs - sb), best);
                    }
                    store_stream(&elem32(outb, r), o);
                }
            };
            if (tl.staged) leftmost(sh.win + tl.off); else leftmost(tl.src);
        }
        if (t < WAVE) {
            const int64_t excl = look_back_resolve(desc, tile, tile_total, err);
            if (t == 0) {
                s_base = excl;
                s_fits = excl + tile_total <= capacity;
                if (tile == ntiles - 1) {
                    offsets[total] = excl + tile_total;
                    *grand = excl + tile_total;
                }
            }
        }
    }
    __syncthreads();

    // 3. offsets and records.  When the tile's records all fit (the normal
    //    case) the stores skip the per-record capacity test.  The leftmost
    //    records and the offsets are written once and not read back here:
    //    streaming stores keep them from displacing the caches' contents
    //    (the next build's rank scatter finds more of its lines cached).
    // The tile's first record and first offset are uniform: stores address
    // them as a scalar base plus a 32-bit lane offset.
    const int64_t base = uniform64(s_base);
    const bool fits = __builtin_amdgcn_readfirstlane(s_fits) != 0;
    E *const rb = recs + base;
    int64_t *const offb = offsets + K0;
    // records this tile may write: all of them when they fit, else those
    // below the capacity
    const int64_t room = capacity - base;
    const uint32_t lim = room <= 0 ? 0u : (room >= int64_t(UINT32_MAX) ? UINT32_MAX : uint32_t(room));
    auto put = [&](uint32_t wo, E rec) {
        if (fits || wo < lim) elem32(rb, wo) = rec;
        else raise_err(err, LRQ_ERR_CAPACITY);
    };
    const int span = int(K1 - K0);
    auto emit = [&](const E *ws) {
        SegRun sr{tl.seg, 0, -1};
#pragma unroll
        for (int j = 0; j < LR_POS; ++j) {
            const int r = j * LR_THREADS + t;
            if (r >= span) break;
            uint32_t wo = s_off[r];
            __builtin_nontemporal_store(base + int64_t(wo), &elem32(offb, r));
            if (A[j] >= 0 && Mk[j] == 0) continue;
            sr.at(segs, K0 + r);
            const P sb = P(sr.sb);
            if (A[j] >= 0) {  // the entries of maximal length, from the mask
                for (uint32_t mk = Mk[j]; mk; mk &= mk - 1) {
                    const E v = ws[A[j] + __ffs(mk) - 1];
                    put(wo++, mkpair<P>(P(v.x - sb), v.y));
                }
            } else {
                const int32_t a = -1 - A[j];
                int32_t a2, z;
                lr_range(sh, tl, r, a2, z);
                P bs, best;
                window_max(ws, a, z, bs, best);
                for (int32_t e = a; e < z; ++e) {
                    const E v = ws[e];
                    if (v.y == best) put(wo++, mkpair<P>(P(v.x - sb), v.y));
                }
            }
        }
    };
    if (tl.staged) emit(sh.win + tl.off); else emit(tl.src);
}

#define LR_ALL_PARAMS(P)                                                                      \
    const pair_t<P> *__restrict__ llrc, const int64_t *__restrict__ blocks, int64_t total,      \
        Segs segs, int64_t *__restrict__ offsets, pair_t<P> *__restrict__ recs,                 \
        int64_t capacity, pair_t<P> *__restrict__ out, uint64_t *desc, uint32_t *ticket,        \
        int64_t *grand, uint32_t *err, int64_t ntiles
#define LR_ALL_FORWARD llrc, blocks, total, segs, offsets, recs, capacity, out, desc, ticket, grand, err, ntiles

// All mode.
template <int LR_TILE>
__global__ __launch_bounds__(LR_THREADS) void lr_all_kernel(LR_ALL_PARAMS(int32_t)) {
    lr_all_tile<LR_TILE, false, int32_t>(LR_ALL_FORWARD);
}

// Both modes in one pass: the leftmost record of every position is written
// while the tile waits for its record offset.
// With 2048-position tiles this kernel fits 80 VGPRs without spills, which
// keeps six waves per SIMD resident (its natural 82 would allow five).
template <int LR_TILE>
constexpr int lr_both_waves() { return LR_TILE == 2048 ? 6 : 1; }

template <int LR_TILE>
__global__ __launch_bounds__(LR_THREADS) __attribute__((amdgpu_waves_per_eu(lr_both_waves<LR_TILE>())))
void lr_both_kernel(LR_ALL_PARAMS(int32_t)) {
    lr_all_tile<LR_TILE, true, int32_t>(LR_ALL_FORWARD);
}

// The same with 64-bit positions and lengths.
template <int LR_TILE>
__global__ __launch_bounds__(LR_THREADS) void lr_all64_kernel(LR_ALL_PARAMS(int64_t)) {
    lr_all_tile<LR_TILE, false, int64_t>(LR_ALL_FORWARD);
}
template <int LR_TILE>
__global__ __launch_bounds__(LR_THREADS) void lr_both64_kernel(LR_ALL_PARAMS(int64_t)) {
    lr_all_tile<LR_TILE, true, int64_t>(LR_ALL_FORWARD);
}
#undef LR_ALL_PARAMS
#undef LR_ALL_FORWARD

// ============================================================================
// Point queries (Algorithm 2 per position; Algorithm 4 for all of them):
// locate the first covering entry of the compact array, then walk right while
// entries start at or before k.  The block table bounds the search: entries
// starting in k's block are [blocks[k/B], blocks[k/B + 1]); the covering ones
// that start earlier are found by a doubling probe backward from blocks[k/B].
// ============================================================================

// The covering window [lo, hi) of global position k in an index (llrc,
// blocks) over `total` positions, the longest length in it, the smallest start
// of that length (global; -1 if the window is empty) and the number of
// entries of that length.
struct PointLR {
    int64_t lo, hi;
    int64_t bs;
    int64_t cnt;
    int64_t best;
};

template <class E>
__device__ __forceinline__ PointLR point_query(const E *__restrict__ llrc,
                                               const int64_t *__restrict__ blocks, int64_t total,
                                               int64_t k) {
    const int64_t m = entry_count(blocks, total);
    const int64_t j = k / LRQ_BLOCK;
    const int64_t first = clamp64(blocks[j], 0, m);
    const int64_t last = clamp64(blocks[j + 1], first, m);
    // lower end: step back from `first` while entries still reach k
    int64_t lo = first, step = 1;
    while (lo > 0 && entry_end(llrc[lo - 1]) >= k) {
        lo = imax(0, lo - step);
        step <<= 1;
    }
    int64_t hi = last;  // answer in [lo, hi]
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (entry_end(llrc[mid]) >= k) hi = mid; else lo = mid + 1;
    }
    PointLR r{lo, lo, -1, 0, 0};
    for (; r.hi < last; ++r.hi) {
        const E v = llrc[r.hi];
        if (v.x > k) break;
        if (v.y > r.best) { r.best = v.y; r.bs = v.x; r.cnt = 1; }
        else if (v.y == r.best) ++r.cnt;
    }
    return r;
}

// Where query q looks: the index buffers, the string's place in the index and
// the global position asked for; ok = false for a string id or position out
// of range.
template <class E>
struct QuerySite {
    const E *llrc;
    const int64_t *blocks;
    int64_t total, begin, k;
    bool ok;
};

// One string: positions of d_pos in [0, n) of the index (llrc, blocks);
// positions, starts and lengths of the type P.
template <class P>
struct OneString {
    using Pos = P;
    using E = pair_t<P>;
    const E *llrc;
    const int64_t *blocks;
    int64_t n;
    __device__ __forceinline__ QuerySite<E> site(int64_t q, const P *pos) const {
        const int64_t k = pos[q];
        return QuerySite<E>{llrc, blocks, n, 0, k, k >= 0 && k < n};
    }
};

// Many resident strings: query q asks for position pos[q] of string sid[q].
struct ManyStrings {
    using Pos = int32_t;
    using E = int2;
    const lrq_string_ref *refs;
    int32_t nrefs;
    const int32_t *sid;
    __device__ __forceinline__ QuerySite<E> site(int64_t q, const int32_t *pos) const {
        const int32_t s = sid[q];
        if (s < 0 || s >= nrefs) return QuerySite<E>{nullptr, nullptr, 0, 0, 0, false};
        const lrq_string_ref r = refs[s];
        const int64_t total = imax(0, imin(r.total, LRQ_MAX_TOTAL));
        const int64_t begin = clamp64(r.begin, 0, total);
        const int64_t len = clamp64(r.length, 0, total - begin);
        const int64_t k = pos[q];
        return QuerySite<E>{reinterpret_cast<const int2 *>(r.llrc), r.blocks, total, begin,
                            begin + k, k >= 0 && k < len};
    }
};

enum { QUERY_LEFTMOST = 0, QUERY_COUNT = 1, QUERY_EMIT = 2 };

// One thread per query.  QUERY_LEFTMOST writes out[q]; QUERY_COUNT writes the
// number of records of q into offsets[q] (scanned into CSR offsets
// afterwards) and, with out, the leftmost record too; QUERY_EMIT writes q's
// records from offsets[q] on, in ascending start, dropping (and flagging)
// those at or beyond capacity.  Starts are local to the queried string.
template <int MODE, class SRC>
__global__ __launch_bounds__(256) void query_kernel(SRC src,
                                                    const typename SRC::Pos *__restrict__ pos,
                                                    int64_t mq, typename SRC::E *__restrict__ out,
                                                    int64_t *__restrict__ offsets,
                                                    typename SRC::E *__restrict__ recs,
                                                    int64_t capacity, uint32_t *err) {
    using P = typename SRC::Pos;
    using E = typename SRC::E;
    const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= mq) return;
    const QuerySite<E> s = src.site(q, pos);
    if (!s.ok) {
        if (MODE != QUERY_EMIT) raise_err(err, LRQ_ERR_QUERY);
        if (out && MODE != QUERY_EMIT) out[q] = mkpair<P>(-1, 0);
        if (MODE == QUERY_COUNT) offsets[q] = 0;
        return;
    }
    const PointLR r = point_query(s.llrc, s.blocks, s.total, s.k);
    if (MODE != QUERY_EMIT && out)
        out[q] = r.bs >= 0 ? mkpair<P>(P(r.bs - s.begin), P(r.best)) : mkpair<P>(-1, 0);
    if (MODE == QUERY_COUNT) offsets[q] = r.cnt;
    if (MODE == QUERY_EMIT && r.cnt > 0) {
        int64_t w = offsets[q];
        for (int64_t e = r.lo; e < r.hi; ++e) {
            const E v = s.llrc[e];
            if (v.y != r.best) continue;
            if (w < capacity) recs[w] = mkpair<P>(P(v.x - s.begin), v.y);
            else raise_err(err, LRQ_ERR_CAPACITY);
            ++w;
        }
    }
}

// Fill `n` 64-bit words with zero (used instead of a memset so that the
// sequence stays a plain kernel chain).
__global__ void zero_words_kernel(uint64_t *p, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        p[i] = 0;
}

// ---- launch timing ------------------------------------------------------------
//
// When enabled (lrq_timing_start), every kernel launch is bracketed by a pair
// of HIP events on its own stream; lrq_timing_collect waits for them and
// returns (kernel name, milliseconds) per launch.  The recorder is per calling
// thread: a thread records its own launches only.

struct TimingRec {
    const char *name;
    hipEvent_t a, b;
};
struct TimingState {
    std::vector<TimingRec> rec;
    size_t n = 0, cap = 0;
    bool on = false;
    std::string only;  // record only this kernel (template arguments aside); empty: all
};
TimingState &timing_state() {
    static thread_local TimingState s;
    return s;
}

bool timing_selected(const TimingState &s, const char *name) {
    if (s.only.empty()) return true;
    const size_t k = s.only.size();
    return std::strncmp(name, s.only.c_str(), k) == 0 && (name[k] == '\0' || name[k] == '<');
}

struct Timed {
    hipStream_t st;
    TimingState &s;
    bool on;
    Timed(const char *name, hipStream_t stream)
        : st(stream), s(timing_state()), on(s.on && s.n < s.cap && timing_selected(s, name)) {
        if (!on) return;
        if (s.n >= s.rec.size()) {
            TimingRec r{name, nullptr, nullptr};
            if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) {
                on = false;
                return;
            }
            s.rec.push_back(r);
        }
        s.rec[s.n].name = name;
        (void)hipEventRecord(s.rec[s.n].a, st);
    }
    ~Timed() {
        if (!on) return;
        (void)hipEventRecord(s.rec[s.n].b, st);
        ++s.n;
    }
};

// Every call site names its stream `st`.
#define LAUNCH(kernel, ...)                                                           \
    do {                                                                            \
        Timed timed_(#kernel, st);                                                  \
        hipLaunchKernelGGL(kernel, __VA_ARGS__);                                    \
    } while (0)

// ---- host helpers -------------------------------------------------------------

int check_launch(const char *what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s: %s", what, hipGetErrorString(e));
        return LRQ_EDEVICE;
    }
    return LRQ_OK;
}

int check_common(int64_t total, const int64_t *seg, int32_t nseg, void *scratch,
                 size_t scratch_bytes, int64_t max_total = LRQ_MAX_TOTAL) {
    if (total < 0) { set_error("total < 0"); return LRQ_EINVAL; }
    if (total > max_total) {
        set_error("total %lld > %s", (long long)total,
                  max_total == LRQ_MAX_TOTAL ? "LRQ_MAX_TOTAL" : "LRQ64_MAX_TOTAL");
        return LRQ_ERANGE;
    }
    if (nseg < 1) { set_error("nseg < 1"); return LRQ_EINVAL; }
    if (!seg && nseg != 1) { set_error("seg_off is NULL but nseg != 1"); return LRQ_EINVAL; }
    if (!scratch) { set_error("scratch is NULL"); return LRQ_EINVAL; }
    if ((reinterpret_cast<uintptr_t>(scratch) & 255) != 0) { set_error("scratch not 256-byte aligned"); return LRQ_EINVAL; }
    const Layout L = layout(total, nseg);
    if (scratch_bytes < L.bytes) {
        set_error("scratch has %zu bytes, needs %zu", scratch_bytes, L.bytes);
        return LRQ_ENOMEM;
    }
    return LRQ_OK;
}

template <class T>
T *at(void *base, size_t off) { return reinterpret_cast<T *>(static_cast<char *>(base) + off); }

unsigned grid_for(int64_t n, int threads) {
    return unsigned((n + threads - 1) / threads);
}

int run_zero(uint64_t *p, int64_t words, hipStream_t st) {
    if (words <= 0) return LRQ_OK;
    const int64_t blocks = (words + 255) / 256;
    LAUNCH(zero_words_kernel, dim3(unsigned(blocks < 1024 ? blocks : 1024)), dim3(256),
                       0, st, p, words);
    return check_launch("zero_words_kernel");
}

bool misaligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) != 0; }

}  // namespace
}  // namespace lrq

// ==== the C ABI =====================================================================

using namespace lrq;

namespace {

int check_index(const void *d_llrc, const int64_t *d_blocks, size_t rec_align = 8) {
    if (!d_llrc || !d_blocks) { set_error("d_llrc / d_llrc_blocks is NULL"); return LRQ_EINVAL; }
    if (misaligned(d_llrc, rec_align) || misaligned(d_blocks, 8)) { set_error("d_llrc / d_llrc_blocks not aligned (%d and 8 bytes)", int(rec_align)); return LRQ_EINVAL; }
    return LRQ_OK;
}

// d_L is written two lengths at a time: l_align bytes (twice its element size).
int check_filter_out(void *d_llrc, int64_t *d_count, int64_t *d_blocks, void *d_L,
                     size_t l_align = 8) {
    if (!d_llrc || !d_count || !d_blocks) { set_error("d_llrc / d_llrc_count / d_llrc_blocks is NULL"); return LRQ_EINVAL; }
    if (misaligned(d_llrc, l_align) || misaligned(d_count, 8) || misaligned(d_blocks, 8)) { set_error("compact-array outputs not aligned (d_llrc to %d bytes, the others to 8)", int(l_align)); return LRQ_EINVAL; }
    if (d_L && misaligned(d_L, l_align)) { set_error("d_L not %d-byte aligned", int(l_align)); return LRQ_EINVAL; }
    return LRQ_OK;
}

// The text's byte values, its code width and (for at most 16 values) the
// packed copy the LCP kernels read.
// cleared: the alphabet mask is already zero (the build path clears it in
// its first kernel).
int pack_text(const uint8_t *d_text, int64_t total, const Layout &L, void *d_scratch,
              hipStream_t st, bool cleared = false) {
    int rc;
    if (!cleared && (rc = run_zero(at<uint64_t>(d_scratch, HDR_ALPHA), 4, st))) return rc;
    // few blocks: every block ends with loads and atomics on the same 32 bytes
    const int64_t words = total >> 3;
    int64_t gb = (words + 4 * 1024 - 1) / (4 * 1024);
    gb = gb < 1 ? 1 : (gb > 256 ? 256 : gb);
    LAUNCH(alpha_kernel, dim3(unsigned(gb)), dim3(1024), 0, st, d_text, total,
           at<uint32_t>(d_scratch, HDR_ALPHA));
    if ((rc = check_launch("alpha_kernel"))) return rc;
    const int64_t pw = packed_words(total);
    int64_t gp = (pw + 255) / 256;
    gp = gp < 1 ? 1 : (gp > 4096 ? 4096 : gp);
    LAUNCH(pack_kernel, dim3(unsigned(gp)), dim3(256), 0, st, d_text, total,
           at<uint32_t>(d_scratch, HDR_ALPHA), at<uint64_t>(d_scratch, L.packed), pw,
           at<int32_t>(d_scratch, HDR_SYM_LG));
    return check_launch("pack_kernel");
}

#define SYM_ARGS(L, scratch) at<uint64_t>(scratch, (L).packed), packed_words(total), \
        at<int32_t>(scratch, HDR_SYM_LG)

template <class P>
int launch_levels(const uint8_t *d_text, int64_t total, const Segs &segs, const pair_t<P> *nbr,
                  const Layout &L, void *d_scratch, hipStream_t st) {
    Levels<P> lv{};
    lv.top = L.levels;
    for (int l = 1; l <= L.levels; ++l) {
        lv.stride[l] = L.stride[l];
        lv.heads[l] = at<pair_t<P>>(d_scratch, L.heads[l]);
    }
    // threads per region: one per level-1 head of the region, at least
    // LEVEL_MIN_THREADS (several waves share the long compares), at most 1024
    int64_t th = L.stride[L.levels] / L.stride[1];
    th = th < LEVEL_MIN_THREADS ? LEVEL_MIN_THREADS : (th > 1024 ? 1024 : th);
    th = (th + 63) / 64 * 64;
    if constexpr (sizeof(P) == 4)
        LAUNCH(plcp_levels_kernel, dim3(unsigned(L.nheads[L.levels])), dim3(unsigned(th)), 0, st,
               d_text, total, segs, nbr, lv, SYM_ARGS(L, d_scratch), at<uint32_t>(d_scratch, HDR_ERR));
    else
        LAUNCH(plcp_levels64_kernel, dim3(unsigned(L.nheads[L.levels])), dim3(unsigned(th)), 0, st,
               d_text, total, segs, nbr, lv, SYM_ARGS(L, d_scratch), at<uint32_t>(d_scratch, HDR_ERR));
    return check_launch("plcp_levels_kernel");
}

int empty_index(int64_t *d_count, int64_t *d_blocks, hipStream_t st) {
    int rc = run_zero(reinterpret_cast<uint64_t *>(d_count), 1, st);
    if (!rc) rc = run_zero(reinterpret_cast<uint64_t *>(d_blocks), 1, st);
    return rc;
}

// Text-order LCP pairs in place over the neighbour pairs; with keepsum, also
// the blocks' keep summaries for llr_bases_kernel.
// d_Lw (32-bit only, optional): the LCP walk writes L there instead of the
// pairs over d_pn.
template <class P>
int plcp_launch(const uint8_t *d_text, int64_t total, const int64_t *d_seg_off, int32_t nseg,
                P *d_pn, void *d_scratch, hipStream_t st, int4 *keepsum,
                bool alpha_cleared = false, int32_t *d_Lw = nullptr) {
    const Segs segs{d_seg_off, nseg, total};
    const Layout L = layout(total, nseg);
    pair_t<P> *pn = reinterpret_cast<pair_t<P> *>(d_pn);
    int rc;
    if ((rc = pack_text(d_text, total, L, d_scratch, st, alpha_cleared))) return rc;
    if ((rc = launch_levels<P>(d_text, total, segs, pn, L, d_scratch, st))) return rc;
    uint32_t *err = at<uint32_t>(d_scratch, HDR_ERR);
    const int64_t blocks = L.plcp_tiles;
    const int chunk = tuning().plcp_chunk;
    if constexpr (sizeof(P) == 4) {
#define PLCP_ARGS dim3(unsigned(blocks)), dim3(PLCP_SPAN / chunk), 0, st, d_text, total, segs, pn, \
        at<int2>(d_scratch, L.heads[1]), L.stride[1], SYM_ARGS(L, d_scratch), err, keepsum
        if (d_Lw) {
            if (chunk == 8) LAUNCH(plcp_chunks_l_kernel<8>, PLCP_ARGS, d_Lw);
            else if (chunk == 32) LAUNCH(plcp_chunks_l_kernel<32>, PLCP_ARGS, d_Lw);
            else LAUNCH(plcp_chunks_l_kernel<16>, PLCP_ARGS, d_Lw);
        } else if (chunk == 8) {
            LAUNCH(plcp_chunks_kernel<8>, PLCP_ARGS);
        } else if (chunk == 32) {
            LAUNCH(plcp_chunks_kernel<32>, PLCP_ARGS);
        } else {
            LAUNCH(plcp_chunks_kernel<16>, PLCP_ARGS);
        }
#undef PLCP_ARGS
    } else {
        (void)keepsum;  // the 64-bit build runs the filter's own look-back
        (void)d_Lw;
#define PLCP_ARGS dim3(unsigned(blocks)), dim3(PLCP_SPAN / chunk), 0, st, d_text, total, segs, pn, \
        at<longlong2>(d_scratch, L.heads[1]), L.stride[1], SYM_ARGS(L, d_scratch), err
        if (chunk == 8) LAUNCH(plcp_chunks64_kernel<8>, PLCP_ARGS);
        else if (chunk == 32) LAUNCH(plcp_chunks64_kernel<32>, PLCP_ARGS);
        else LAUNCH(plcp_chunks64_kernel<16>, PLCP_ARGS);
#undef PLCP_ARGS
    }
    return check_launch("plcp_chunks_kernel");
}

// tile_base: exclusive compact-array bases per PLCP_SPAN block (from
// llr_bases_kernel), or null for the look-back.
// from_L (32-bit only): d_pn holds L (int32[total]) rather than pairs.
template <class P>
int filter_launch(const P *d_pn, int64_t total, const int64_t *d_seg_off, int32_t nseg,
                  void *d_llrc, int64_t *d_count, int64_t *d_blocks, P *d_L,
                  void *d_scratch, hipStream_t st, const int64_t *tile_base = nullptr,
                  bool from_L = false) {
    const Layout L = layout(total, nseg);
    uint64_t *state = at<uint64_t>(d_scratch, L.llr_state);
    if (!tile_base) {
        int rc = run_zero(state, 1 + L.llr_tiles, st);
        if (rc) return rc;
    }
    const Segs segs{d_seg_off, nseg, total};
#define LLR_ARGS dim3(unsigned(L.llr_tiles)), dim3(64 * tuning().llr_waves), 0, st,              \
        reinterpret_cast<const pair_t<P> *>(d_pn), total, segs,                                 \
        reinterpret_cast<pair_t<P> *>(d_llrc), d_count, d_blocks, d_L, state + 1,               \
        reinterpret_cast<uint32_t *>(state), at<uint32_t>(d_scratch, HDR_ERR), L.llr_tiles,    \
        tile_base
    if constexpr (sizeof(P) == 4) {
        if (from_L) {
            if (tuning().llr_waves == 8) LAUNCH(llr_filter_l_kernel<8>, LLR_ARGS);
            else LAUNCH(llr_filter_l_kernel<4>, LLR_ARGS);
        } else if (tuning().llr_waves == 8) {
            LAUNCH(llr_filter_kernel<8>, LLR_ARGS);
        } else {
            LAUNCH(llr_filter_kernel<4>, LLR_ARGS);
        }
    } else {
        if (tuning().llr_waves == 8) LAUNCH(llr_filter64_kernel<8>, LLR_ARGS);
        else LAUNCH(llr_filter64_kernel<4>, LLR_ARGS);
    }
#undef LLR_ARGS
    return check_launch("llr_filter_kernel");
}

}  // namespace

namespace lrq {
namespace {

// The calls with 32-bit (lrq_) and 64-bit (lrq64_) positions share these
// bodies; max_total is the size limit of each family.

// Threads per rank-scatter block.  Each block waits for one segment search
// by its first wave; with at most 64 strings the search is one round and
// larger blocks pay (16.8M-character string: 268 -> 219 us with 512), while a
// batch of 512 strings (two rounds) is faster with 256 (951 against 993 us).
inline unsigned rs_threads(int32_t nseg) { return nseg > WAVE ? 256u : 512u; }

template <class P>
int rank_scatter_impl(const P *d_sa, int64_t total, const int64_t *d_seg_off, int32_t nseg,
                      P *d_nbr, P *d_rank, void *d_scratch, size_t scratch_bytes, void *stream,
                      int64_t max_total) {
    int rc = check_common(total, d_seg_off, nseg, d_scratch, scratch_bytes, max_total);
    if (rc) return rc;
    if (total == 0) return LRQ_OK;
    if (!d_sa || !d_nbr) { set_error("d_sa / d_nbr is NULL"); return LRQ_EINVAL; }
    if (misaligned(d_nbr, 2 * sizeof(P))) { set_error("d_nbr not %d-byte aligned", int(2 * sizeof(P))); return LRQ_EINVAL; }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Segs segs{d_seg_off, nseg, total};
    if constexpr (sizeof(P) == 4)
        LAUNCH(rank_scatter_kernel, dim3(grid_for(total, rs_threads(nseg))),
               dim3(rs_threads(nseg)), 0, st, d_sa, total, segs, reinterpret_cast<int2 *>(d_nbr), d_rank,
               at<uint32_t>(d_scratch, HDR_ERR), nullptr, 0);
    else
        LAUNCH(rank_scatter64_kernel, dim3(grid_for(total, rs_threads(nseg))),
               dim3(rs_threads(nseg)), 0, st, d_sa, total, segs, reinterpret_cast<longlong2 *>(d_nbr), d_rank,
               at<uint32_t>(d_scratch, HDR_ERR), nullptr, 0);
    return check_launch("rank_scatter_kernel");
}

template <class P>
int plcp_impl(const uint8_t *d_text, int64_t total, const int64_t *d_seg_off, int32_t nseg,
              P *d_pn, void *d_scratch, size_t scratch_bytes, void *stream, int64_t max_total) {
    int rc = check_common(total, d_seg_off, nseg, d_scratch, scratch_bytes, max_total);
    if (rc) return rc;
    if (total == 0) return LRQ_OK;
    if (!d_text || !d_pn) { set_error("d_text / d_pn is NULL"); return LRQ_EINVAL; }
    if (misaligned(d_text, 8)) { set_error("d_text not 8-byte aligned"); return LRQ_EINVAL; }
    if (misaligned(d_pn, 2 * sizeof(P))) { set_error("d_pn not %d-byte aligned", int(2 * sizeof(P))); return LRQ_EINVAL; }
    return plcp_launch<P>(d_text, total, d_seg_off, nseg, d_pn, d_scratch,
                          static_cast<hipStream_t>(stream), nullptr);
}

template <class P>
int filter_impl(const P *d_pn, int64_t total, const int64_t *d_seg_off, int32_t nseg,
                void *d_llrc, int64_t *d_llrc_count, int64_t *d_llrc_blocks, P *d_L,
                void *d_scratch, size_t scratch_bytes, void *stream, int64_t max_total) {
    int rc = check_common(total, d_seg_off, nseg, d_scratch, scratch_bytes, max_total);
    if (rc) return rc;
    if ((rc = check_filter_out(d_llrc, d_llrc_count, d_llrc_blocks, d_L, 2 * sizeof(P)))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (total == 0) return empty_index(d_llrc_count, d_llrc_blocks, st);
    if (!d_pn) { set_error("d_pn is NULL"); return LRQ_EINVAL; }
    if (misaligned(d_pn, 16)) { set_error("d_pn not 16-byte aligned"); return LRQ_EINVAL; }
    return filter_launch<P>(d_pn, total, d_seg_off, nseg, d_llrc, d_llrc_count, d_llrc_blocks,
                            d_L, d_scratch, st);
}

template <class P>
int index_build_impl(const uint8_t *d_text, const P *d_sa, int64_t total,
                     const int64_t *d_seg_off, int32_t nseg, P *d_work, void *d_llrc,
                     int64_t *d_llrc_count, int64_t *d_llrc_blocks, P *d_L, void *d_scratch,
                     size_t scratch_bytes, void *stream, int64_t max_total) {
    int rc = check_common(total, d_seg_off, nseg, d_scratch, scratch_bytes, max_total);
    if (rc) return rc;
    if ((rc = check_filter_out(d_llrc, d_llrc_count, d_llrc_blocks, d_L, 2 * sizeof(P)))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (total == 0) return empty_index(d_llrc_count, d_llrc_blocks, st);
    if (!d_text || !d_sa || !d_work) { set_error("d_text / d_sa / d_work is NULL"); return LRQ_EINVAL; }
    if (misaligned(d_work, 16)) { set_error("d_work not 16-byte aligned"); return LRQ_EINVAL; }
    if (misaligned(d_text, 8)) { set_error("d_text not 8-byte aligned"); return LRQ_EINVAL; }
    // The unfused 32-bit build keeps the neighbour pairs in the compact
    // array's buffer (its n entries are as large as the pairs, and the filter
    // overwrites them only after the LCP walk has read them), and the walk
    // writes L alone into d_L, or else into the first half of d_work: the
    // filter then reads 4 bytes per position instead of 8.
    const bool l_only = sizeof(P) == 4 && !tuning().fuse_filter;
    P *nbr_buf = l_only ? reinterpret_cast<P *>(d_llrc) : d_work;
    int32_t *l_buf = reinterpret_cast<int32_t *>(d_L ? d_L : d_work);
    {
        // the rank scatter's block 0 also clears the alphabet mask
        const Segs segs{d_seg_off, nseg, total};
        if constexpr (sizeof(P) == 4)
            LAUNCH(rank_scatter_kernel, dim3(grid_for(total, rs_threads(nseg))),
                   dim3(rs_threads(nseg)), 0, st, d_sa, total, segs, reinterpret_cast<int2 *>(nbr_buf), nullptr,
                   at<uint32_t>(d_scratch, HDR_ERR), at<uint64_t>(d_scratch, HDR_ALPHA), 4);
        else
            LAUNCH(rank_scatter64_kernel, dim3(grid_for(total, rs_threads(nseg))),
                   dim3(rs_threads(nseg)), 0, st, d_sa, total, segs, reinterpret_cast<longlong2 *>(d_work), nullptr,
                   at<uint32_t>(d_scratch, HDR_ERR), at<uint64_t>(d_scratch, HDR_ALPHA), 4);
        if ((rc = check_launch("rank_scatter_kernel"))) return rc;
    }
    const Layout L = layout(total, nseg);
    if constexpr (sizeof(P) == 8) {
        // 64-bit: LCP pairs, then the filter with its own look-back
        if ((rc = plcp_launch<P>(d_text, total, d_seg_off, nseg, d_work, d_scratch, st, nullptr,
                                 true)))
            return rc;
        return filter_launch<P>(d_work, total, d_seg_off, nseg, d_llrc, d_llrc_count,
                                d_llrc_blocks, d_L, d_scratch, st);
    } else {
        if (!tuning().fuse_filter) {
            // Text-order LCP with per-block keep counts, their scan, then the
            // filter at known bases (no look-back).
            uint64_t *state = at<uint64_t>(d_scratch, L.plcp_state);
            int4 *keepsum = reinterpret_cast<int4 *>(state + 2);
            int64_t *bases = reinterpret_cast<int64_t *>(state + 2 + 2 * L.plcp_tiles);
            if ((rc = plcp_launch<P>(d_text, total, d_seg_off, nseg, nbr_buf, d_scratch, st,
                                     keepsum, true, l_buf)))
                return rc;
            LAUNCH(llr_bases_kernel, dim3(1), dim3(BASES_THREADS), 0, st, keepsum, L.plcp_tiles,
                   bases, total, d_llrc_count, d_llrc_blocks);
            if ((rc = check_launch("llr_bases_kernel"))) return rc;
            return filter_launch<P>(reinterpret_cast<const P *>(l_buf), total, d_seg_off, nseg,
                                    d_llrc, d_llrc_count, d_llrc_blocks, nullptr, d_scratch, st,
                                    bases, true);
        }
        // text-order LCP fused with the LLR filter
        const Segs segs{d_seg_off, nseg, total};
        const int2 *nbr = reinterpret_cast<const int2 *>(d_work);
        if ((rc = pack_text(d_text, total, L, d_scratch, st, true))) return rc;
        if ((rc = launch_levels<int32_t>(d_text, total, segs, nbr, L, d_scratch, st))) return rc;
        uint64_t *state = at<uint64_t>(d_scratch, L.plcp_state);
        if ((rc = run_zero(state, 1 + L.plcp_tiles, st))) return rc;
        const int chunk = tuning().plcp_chunk;
#define FUSED_ARGS dim3(unsigned(L.plcp_tiles)), dim3(PLCP_SPAN / chunk), 0, st, d_text, total,   \
        segs, nbr, at<int2>(d_scratch, L.heads[1]), L.stride[1],                               \
        reinterpret_cast<int2 *>(d_llrc), d_llrc_count, d_llrc_blocks, d_L, state + 1,         \
        reinterpret_cast<uint32_t *>(state), SYM_ARGS(L, d_scratch),                           \
        at<uint32_t>(d_scratch, HDR_ERR), L.plcp_tiles
        if (chunk == 8) LAUNCH(plcp_llr_kernel<8>, FUSED_ARGS);
        else if (chunk == 32) LAUNCH(plcp_llr_kernel<32>, FUSED_ARGS);
        else LAUNCH(plcp_llr_kernel<16>, FUSED_ARGS);
#undef FUSED_ARGS
        return check_launch("plcp_llr_kernel");
    }
}

template <class P>
int lr_leftmost_impl(const void *d_llrc, const int64_t *d_llrc_blocks, int64_t total,
                     const int64_t *d_seg_off, int32_t nseg, void *d_out, void *d_scratch,
                     size_t scratch_bytes, void *stream, int64_t max_total) {
    int rc = check_common(total, d_seg_off, nseg, d_scratch, scratch_bytes, max_total);
    if (rc) return rc;
    if (total == 0) return LRQ_OK;
    if ((rc = check_index(d_llrc, d_llrc_blocks, 2 * sizeof(P)))) return rc;
    if (!d_out || misaligned(d_out, 16)) { set_error("d_out NULL or not 16-byte aligned"); return LRQ_EINVAL; }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Segs segs{d_seg_off, nseg, total};
    const Layout L = layout(total, nseg);
#define LR_ARGS dim3(unsigned(L.lr_tiles)), dim3(LR_THREADS), 0, st,                            \
        reinterpret_cast<const pair_t<P> *>(d_llrc), d_llrc_blocks, total, segs,               \
        reinterpret_cast<pair_t<P> *>(d_out)
    if constexpr (sizeof(P) == 4) {
        switch (tuning().lr_tile) {
            case 1024: LAUNCH(lr_leftmost_kernel<1024>, LR_ARGS); break;
            case 4096: LAUNCH(lr_leftmost_kernel<4096>, LR_ARGS); break;
            default: LAUNCH(lr_leftmost_kernel<2048>, LR_ARGS); break;
        }
    } else {
        switch (tuning().lr_tile) {
            case 1024: LAUNCH(lr_leftmost64_kernel<1024>, LR_ARGS); break;
            case 4096: LAUNCH(lr_leftmost64_kernel<4096>, LR_ARGS); break;
            default: LAUNCH(lr_leftmost64_kernel<2048>, LR_ARGS); break;
        }
    }
#undef LR_ARGS
    return check_launch("lr_leftmost_kernel");
}

int read_total(int64_t *h_total, const int64_t *d_val, hipStream_t st) {
    hipError_t e = hipMemcpyAsync(h_total, d_val, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) { set_error("reading the record total: %s", hipGetErrorString(e)); return LRQ_EDEVICE; }
    return LRQ_OK;
}

template <class P>
int lr_all_count_impl(const void *d_llrc, const int64_t *d_llrc_blocks, int64_t total,
                      const int64_t *d_seg_off, int32_t nseg, int64_t *h_total, void *d_scratch,
                      size_t scratch_bytes, void *stream, int64_t max_total) {
    int rc = check_common(total, d_seg_off, nseg, d_scratch, scratch_bytes, max_total);
    if (rc) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    int64_t *grand = at<int64_t>(d_scratch, HDR_ALL_TOTAL);
    if ((rc = run_zero(reinterpret_cast<uint64_t *>(grand), 1, st))) return rc;
    if (total > 0) {
        if ((rc = check_index(d_llrc, d_llrc_blocks, 2 * sizeof(P)))) return rc;
        const Segs segs{d_seg_off, nseg, total};
        const Layout L = layout(total, nseg);
#define LR_ARGS dim3(unsigned(L.lr_tiles)), dim3(LR_THREADS), 0, st,                            \
        reinterpret_cast<const pair_t<P> *>(d_llrc), d_llrc_blocks, total, segs,               \
        reinterpret_cast<unsigned long long *>(grand)
        if constexpr (sizeof(P) == 4) {
            switch (tuning().lr_tile) {
                case 1024: LAUNCH(lr_all_count_kernel<1024>, LR_ARGS); break;
                case 4096: LAUNCH(lr_all_count_kernel<4096>, LR_ARGS); break;
                default: LAUNCH(lr_all_count_kernel<2048>, LR_ARGS); break;
            }
        } else {
            switch (tuning().lr_tile) {
                case 1024: LAUNCH(lr_all_count64_kernel<1024>, LR_ARGS); break;
                case 4096: LAUNCH(lr_all_count64_kernel<4096>, LR_ARGS); break;
                default: LAUNCH(lr_all_count64_kernel<2048>, LR_ARGS); break;
            }
        }
#undef LR_ARGS
        if ((rc = check_launch("lr_all_count_kernel"))) return rc;
    }
    return h_total ? read_total(h_total, grand, st) : LRQ_OK;
}

template <class P>
int lr_all_run(const void *d_llrc, const int64_t *d_llrc_blocks, int64_t total,
               const int64_t *d_seg_off, int32_t nseg, void *d_out, int64_t *d_offsets,
               void *d_recs, int64_t capacity, int64_t *h_total, void *d_scratch,
               size_t scratch_bytes, void *stream, int64_t max_total) {
    int rc = check_common(total, d_seg_off, nseg, d_scratch, scratch_bytes, max_total);
    if (rc) return rc;
    if (!d_offsets || misaligned(d_offsets, 16)) { set_error("d_offsets NULL or not 16-byte aligned"); return LRQ_EINVAL; }
    if (capacity < 0 || (capacity > 0 && (!d_recs || misaligned(d_recs, 2 * sizeof(P))))) { set_error("bad d_recs / capacity"); return LRQ_EINVAL; }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Layout L = layout(total, nseg);
    int64_t *grand = at<int64_t>(d_scratch, HDR_ALL_TOTAL);
    if (total == 0) {
        if ((rc = run_zero(reinterpret_cast<uint64_t *>(d_offsets), 1, st))) return rc;
        if ((rc = run_zero(reinterpret_cast<uint64_t *>(grand), 1, st))) return rc;
    } else {
        if ((rc = check_index(d_llrc, d_llrc_blocks, 2 * sizeof(P)))) return rc;
        uint64_t *state = at<uint64_t>(d_scratch, L.lr_state);
        if ((rc = run_zero(state, 1 + L.lr_tiles, st))) return rc;
        const Segs segs{d_seg_off, nseg, total};
#define LR_ARGS dim3(unsigned(L.lr_tiles)), dim3(LR_THREADS), 0, st,                            \
        reinterpret_cast<const pair_t<P> *>(d_llrc), d_llrc_blocks, total, segs, d_offsets,    \
        reinterpret_cast<pair_t<P> *>(d_recs), capacity, reinterpret_cast<pair_t<P> *>(d_out), \
        state + 1, reinterpret_cast<uint32_t *>(state), grand, at<uint32_t>(d_scratch, HDR_ERR), \
        L.lr_tiles
        if constexpr (sizeof(P) == 4) {
            if (d_out) {
                switch (tuning().lr_tile) {
                    case 1024: LAUNCH(lr_both_kernel<1024>, LR_ARGS); break;
                    case 4096: LAUNCH(lr_both_kernel<4096>, LR_ARGS); break;
                    default: LAUNCH(lr_both_kernel<2048>, LR_ARGS); break;
                }
            } else {
                switch (tuning().lr_tile) {
                    case 1024: LAUNCH(lr_all_kernel<1024>, LR_ARGS); break;
                    case 4096: LAUNCH(lr_all_kernel<4096>, LR_ARGS); break;
                    default: LAUNCH(lr_all_kernel<2048>, LR_ARGS); break;
                }
            }
        } else {
            if (d_out) {
                switch (tuning().lr_tile) {
                    case 1024: LAUNCH(lr_both64_kernel<1024>, LR_ARGS); break;
                    case 4096: LAUNCH(lr_both64_kernel<4096>, LR_ARGS); break;
                    default: LAUNCH(lr_both64_kernel<2048>, LR_ARGS); break;
                }
            } else {
                switch (tuning().lr_tile) {
                    case 1024: LAUNCH(lr_all64_kernel<1024>, LR_ARGS); break;
                    case 4096: LAUNCH(lr_all64_kernel<4096>, LR_ARGS); break;
                    default: LAUNCH(lr_all64_kernel<2048>, LR_ARGS); break;
                }
            }
        }
#undef LR_ARGS
        if ((rc = check_launch(d_out ? "lr_both_kernel" : "lr_all_kernel"))) return rc;
    }
    if (!h_total) return LRQ_OK;
    if ((rc = read_total(h_total, grand, st))) return rc;
    if (*h_total > capacity) {
        set_error("%lld records, capacity %lld", (long long)*h_total, (long long)capacity);
        return LRQ_ENOSPC;
    }
    return LRQ_OK;
}

}  // namespace
}  // namespace lrq

extern "C" {

int lrq_rank_scatter(const int32_t *d_sa, int64_t total, const int64_t *d_seg_off, int32_t nseg,
                     int32_t *d_nbr, int32_t *d_rank, void *d_scratch, size_t scratch_bytes,
                     void *stream) {
    clear_error();
    return rank_scatter_impl<int32_t>(d_sa, total, d_seg_off, nseg, d_nbr, d_rank, d_scratch,
                                      scratch_bytes, stream, LRQ_MAX_TOTAL);
}

int lrq_plcp(const uint8_t *d_text, int64_t total, const int64_t *d_seg_off, int32_t nseg,
             int32_t *d_pn, void *d_scratch, size_t scratch_bytes, void *stream) {
    clear_error();
    return plcp_impl<int32_t>(d_text, total, d_seg_off, nseg, d_pn, d_scratch, scratch_bytes,
                              stream, LRQ_MAX_TOTAL);
}

int lrq_llr_filter(const int32_t *d_pn, int64_t total, const int64_t *d_seg_off, int32_t nseg,
                   lrq_rec *d_llrc, int64_t *d_llrc_count, int64_t *d_llrc_blocks, int32_t *d_L,
                   void *d_scratch, size_t scratch_bytes, void *stream) {
    clear_error();
    return filter_impl<int32_t>(d_pn, total, d_seg_off, nseg, d_llrc, d_llrc_count,
                                d_llrc_blocks, d_L, d_scratch, scratch_bytes, stream,
                                LRQ_MAX_TOTAL);
}

int lrq_llr_from_rank_lcp(const int32_t *d_rank, const int32_t *d_lcp, int64_t n, int32_t *d_work,
                          lrq_rec *d_llrc, int64_t *d_llrc_count, int64_t *d_llrc_blocks,
                          int32_t *d_L, void *d_scratch, size_t scratch_bytes, void *stream) {
    clear_error();
    int rc = check_common(n, nullptr, 1, d_scratch, scratch_bytes);
    if (rc) return rc;
    if ((rc = check_filter_out(d_llrc, d_llrc_count, d_llrc_blocks, d_L, 8))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n == 0) return empty_index(d_llrc_count, d_llrc_blocks, st);
    if (!d_rank || !d_lcp || !d_work) { set_error("d_rank / d_lcp / d_work is NULL"); return LRQ_EINVAL; }
    if (misaligned(d_work, 16)) { set_error("d_work not 16-byte aligned"); return LRQ_EINVAL; }
    LAUNCH(gather_rank_lcp_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, d_rank, d_lcp, n,
           reinterpret_cast<int2 *>(d_work), at<uint32_t>(d_scratch, HDR_ERR));
    if ((rc = check_launch("gather_rank_lcp_kernel"))) return rc;
    return filter_launch<int32_t>(d_work, n, nullptr, 1, d_llrc, d_llrc_count, d_llrc_blocks, d_L,
                                  d_scratch, st);
}

int lrq_index_build(const uint8_t *d_text, const int32_t *d_sa, int64_t total,
                    const int64_t *d_seg_off, int32_t nseg, int32_t *d_work, lrq_rec *d_llrc,
                    int64_t *d_llrc_count, int64_t *d_llrc_blocks, int32_t *d_L, void *d_scratch,
                    size_t scratch_bytes, void *stream) {
    clear_error();
    return index_build_impl<int32_t>(d_text, d_sa, total, d_seg_off, nseg, d_work, d_llrc,
                                     d_llrc_count, d_llrc_blocks, d_L, d_scratch, scratch_bytes,
                                     stream, LRQ_MAX_TOTAL);
}

int lrq_lr_leftmost(const lrq_rec *d_llrc, const int64_t *d_llrc_blocks, int64_t total,
                    const int64_t *d_seg_off, int32_t nseg, lrq_rec *d_out, void *d_scratch,
                    size_t scratch_bytes, void *stream) {
    clear_error();
    return lr_leftmost_impl<int32_t>(d_llrc, d_llrc_blocks, total, d_seg_off, nseg, d_out,
                                     d_scratch, scratch_bytes, stream, LRQ_MAX_TOTAL);
}

int lrq_lr_all_count(const lrq_rec *d_llrc, const int64_t *d_llrc_blocks, int64_t total,
                     const int64_t *d_seg_off, int32_t nseg, int64_t *h_total, void *d_scratch,
                     size_t scratch_bytes, void *stream) {
    clear_error();
    return lr_all_count_impl<int32_t>(d_llrc, d_llrc_blocks, total, d_seg_off, nseg, h_total,
                                      d_scratch, scratch_bytes, stream, LRQ_MAX_TOTAL);
}

int lrq_lr_all(const lrq_rec *d_llrc, const int64_t *d_llrc_blocks, int64_t total,
               const int64_t *d_seg_off, int32_t nseg, int64_t *d_offsets, lrq_rec *d_recs,
               int64_t capacity, int64_t *h_total, void *d_scratch, size_t scratch_bytes,
               void *stream) {
    clear_error();
    return lr_all_run<int32_t>(d_llrc, d_llrc_blocks, total, d_seg_off, nseg, nullptr, d_offsets,
                               d_recs, capacity, h_total, d_scratch, scratch_bytes, stream,
                               LRQ_MAX_TOTAL);
}

int lrq_lr_both(const lrq_rec *d_llrc, const int64_t *d_llrc_blocks, int64_t total,
                const int64_t *d_seg_off, int32_t nseg, lrq_rec *d_out, int64_t *d_offsets,
                lrq_rec *d_recs, int64_t capacity, int64_t *h_total, void *d_scratch,
                size_t scratch_bytes, void *stream) {
    clear_error();
    if (total > 0 && (!d_out || misaligned(d_out, 8))) {
        set_error("d_out NULL or not 8-byte aligned");
        return LRQ_EINVAL;
    }
    return lr_all_run<int32_t>(d_llrc, d_llrc_blocks, total, d_seg_off, nseg,
                               total > 0 ? d_out : nullptr, d_offsets, d_recs, capacity, h_total,
                               d_scratch, scratch_bytes, stream, LRQ_MAX_TOTAL);
}

// ---- 64-bit positions and lengths --------------------------------------------

int lrq64_rank_scatter(const int64_t *d_sa, int64_t total, const int64_t *d_seg_off,
                       int32_t nseg, int64_t *d_nbr, int64_t *d_rank, void *d_scratch,
                       size_t scratch_bytes, void *stream) {
    clear_error();
    return rank_scatter_impl<int64_t>(d_sa, total, d_seg_off, nseg, d_nbr, d_rank, d_scratch,
                                      scratch_bytes, stream, LRQ64_MAX_TOTAL);
}

int lrq64_plcp(const uint8_t *d_text, int64_t total, const int64_t *d_seg_off, int32_t nseg,
               int64_t *d_pn, void *d_scratch, size_t scratch_bytes, void *stream) {
    clear_error();
    return plcp_impl<int64_t>(d_text, total, d_seg_off, nseg, d_pn, d_scratch, scratch_bytes,
                              stream, LRQ64_MAX_TOTAL);
}

int lrq64_llr_filter(const int64_t *d_pn, int64_t total, const int64_t *d_seg_off, int32_t nseg,
                     lrq_rec64 *d_llrc, int64_t *d_llrc_count, int64_t *d_llrc_blocks,
                     int64_t *d_L, void *d_scratch, size_t scratch_bytes, void *stream) {
    clear_error();
    return filter_impl<int64_t>(d_pn, total, d_seg_off, nseg, d_llrc, d_llrc_count,
                                d_llrc_blocks, d_L, d_scratch, scratch_bytes, stream,
                                LRQ64_MAX_TOTAL);
}

int lrq64_index_build(const uint8_t *d_text, const int64_t *d_sa, int64_t total,
                      const int64_t *d_seg_off, int32_t nseg, int64_t *d_work, lrq_rec64 *d_llrc,
                      int64_t *d_llrc_count, int64_t *d_llrc_blocks, int64_t *d_L,
                      void *d_scratch, size_t scratch_bytes, void *stream) {
    clear_error();
    return index_build_impl<int64_t>(d_text, d_sa, total, d_seg_off, nseg, d_work, d_llrc,
                                     d_llrc_count, d_llrc_blocks, d_L, d_scratch, scratch_bytes,
                                     stream, LRQ64_MAX_TOTAL);
}

int lrq64_lr_leftmost(const lrq_rec64 *d_llrc, const int64_t *d_llrc_blocks, int64_t total,
                      const int64_t *d_seg_off, int32_t nseg, lrq_rec64 *d_out, void *d_scratch,
                      size_t scratch_bytes, void *stream) {
    clear_error();
    return lr_leftmost_impl<int64_t>(d_llrc, d_llrc_blocks, total, d_seg_off, nseg, d_out,
                                     d_scratch, scratch_bytes, stream, LRQ64_MAX_TOTAL);
}

int lrq64_lr_all_count(const lrq_rec64 *d_llrc, const int64_t *d_llrc_blocks, int64_t total,
                       const int64_t *d_seg_off, int32_t nseg, int64_t *h_total, void *d_scratch,
                       size_t scratch_bytes, void *stream) {
    clear_error();
    return lr_all_count_impl<int64_t>(d_llrc, d_llrc_blocks, total, d_seg_off, nseg, h_total,
                                      d_scratch, scratch_bytes, stream, LRQ64_MAX_TOTAL);
}

int lrq64_lr_all(const lrq_rec64 *d_llrc, const int64_t *d_llrc_blocks, int64_t total,
                 const int64_t *d_seg_off, int32_t nseg, int64_t *d_offsets, lrq_rec64 *d_recs,
                 int64_t capacity, int64_t *h_total, void *d_scratch, size_t scratch_bytes,
                 void *stream) {
    clear_error();
    return lr_all_run<int64_t>(d_llrc, d_llrc_blocks, total, d_seg_off, nseg, nullptr, d_offsets,
                               d_recs, capacity, h_total, d_scratch, scratch_bytes, stream,
                               LRQ64_MAX_TOTAL);
}

int lrq64_lr_both(const lrq_rec64 *d_llrc, const int64_t *d_llrc_blocks, int64_t total,
                  const int64_t *d_seg_off, int32_t nseg, lrq_rec64 *d_out, int64_t *d_offsets,
                  lrq_rec64 *d_recs, int64_t capacity, int64_t *h_total, void *d_scratch,
                  size_t scratch_bytes, void *stream) {
    clear_error();
    if (total > 0 && (!d_out || misaligned(d_out, 16))) {
        set_error("d_out NULL or not 16-byte aligned");
        return LRQ_EINVAL;
    }
    return lr_all_run<int64_t>(d_llrc, d_llrc_blocks, total, d_seg_off, nseg,
                               total > 0 ? d_out : nullptr, d_offsets, d_recs, capacity, h_total,
                               d_scratch, scratch_bytes, stream, LRQ64_MAX_TOTAL);
}

int lrq_read_errors(void *d_scratch, uint32_t *h_flags, void *stream) {
    clear_error();
    if (!d_scratch || !h_flags) { set_error("NULL argument"); return LRQ_EINVAL; }
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint32_t *err = at<uint32_t>(d_scratch, HDR_ERR);
    hipError_t e = hipMemcpyAsync(h_flags, err, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) { set_error("reading error word: %s", hipGetErrorString(e)); return LRQ_EDEVICE; }
    return run_zero(reinterpret_cast<uint64_t *>(err), 1, st);
}

int lrq_timing_start(int32_t max_records) {
    clear_error();
    if (max_records < 0) { set_error("max_records < 0"); return LRQ_EINVAL; }
    TimingState &s = timing_state();
    s.n = 0;
    s.cap = size_t(max_records);
    s.on = max_records > 0;
    return LRQ_OK;
}

int lrq_timing_only(const char *kernel) {
    clear_error();
    timing_state().only = kernel ? kernel : "";
    return LRQ_OK;
}

int lrq_timing_collect(int32_t cap, const char **names, float *ms, int32_t *count) {
    clear_error();
    if (!count || (cap > 0 && (!names || !ms))) { set_error("NULL argument"); return LRQ_EINVAL; }
    TimingState &s = timing_state();
    s.on = false;
    const size_t n = s.n;
    int rc = LRQ_OK;
    for (size_t i = 0; i < n && int64_t(i) < int64_t(cap); ++i) {
        float t = 0.f;
        hipError_t e = hipEventSynchronize(s.rec[i].b);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, s.rec[i].a, s.rec[i].b);
        if (e != hipSuccess) { set_error("timing event: %s", hipGetErrorString(e)); rc = LRQ_EDEVICE; }
        names[i] = s.rec[i].name;
        ms[i] = t;
    }
    *count = int32_t(n);
    s.n = 0;
    return rc;
}

}  // extern "C"

// ============================================================================
// Suffix arrays on the device: prefix doubling (Manber and Myers, "Suffix
// arrays: a new method for on-line string searches", SIAM J. Comput. 1993)
// over a least-significant-digit radix sort of 64-bit keys written for this
// library.  Round 0 sorts every suffix by its first K characters -- an
// order-preserving code of the byte values present, 0 past the string's end --
// with its string's index in the top bits.  Round r sorts by (rank of the first
// h characters, rank of the next h characters), h = K 2^(r-1), until all ranks
// differ.  Ranks are dense (the number of distinct keys before), so a key is
// below (groups + 1)^2 and the sort only visits the bits it needs.
// ============================================================================

namespace lrq {
namespace {

constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;
constexpr int64_t RS_TILE = RS_THREADS * RS_ITEMS;  // elements per radix / scan tile

// Round-0 keys.  code[c] = 1 + (number of present byte values below c).
__global__ __launch_bounds__(RS_THREADS) void sa_key0_kernel(
    const uint8_t *__restrict__ text, int64_t total, Segs segs, const uint32_t *__restrict__ mask,
    int cb, int K, int sbits, uint64_t *__restrict__ keys, int32_t *__restrict__ vals) {
    __shared__ uint16_t code[256];  // up to 256: one more than a byte holds
    __shared__ int32_t s_b;
    const int t = threadIdx.x;
    {
        int32_t below = 0;
        for (int q = 0; q < (t >> 5); ++q) below += __popc(mask[q]);
        below += __popc(mask[t >> 5] & ((1u << (t & 31)) - 1u));
        code[t] = uint16_t(below + 1);
    }
    const int64_t i0 = int64_t(blockIdx.x) * RS_THREADS;
    int32_t b = block_segment(segs, imin(i0, total - 1), &s_b);  // includes the barrier
    const int64_t i = i0 + t;
    if (i >= total) return;
    b = segs.advance(b, i);
    const int64_t e = segs.end(b);
    const int top = 64 - sbits;
    uint64_t key = sbits ? uint64_t(b) << top : 0;
    for (int q = 0; q < K; ++q) {
        const int64_t x = i + q;
        if (x >= e) break;
        key |= uint64_t(code[text[x]]) << (top - cb * (q + 1));
    }
    keys[i] = key;
    vals[i] = int32_t(i);
}

// Per-tile digit counts: hist[digit * ntiles + tile].
__global__ __launch_bounds__(RS_THREADS) void rs_hist_kernel(const uint64_t *__restrict__ keys,
                                                             int64_t n, int shift,
                                                             uint32_t *__restrict__ hist,
                                                             int64_t ntiles) {
    __shared__ uint32_t h[256];
    const int t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const int64_t base = int64_t(blockIdx.x) * RS_TILE;
    uint32_t d[RS_ITEMS];
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const int64_t idx = base + int64_t(j) * RS_THREADS + t;
        d[j] = idx < n ? uint32_t(keys[idx] >> shift) & 255u : 256u;
    }
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j)
        if (d[j] < 256u) atomicAdd(&h[d[j]], 1u);
    __syncthreads();
    hist[int64_t(t) * ntiles + blockIdx.x] = h[t];
}

// Exclusive scan (uint32 or int64) in three launches: tile sums, one block
// over the sums, tiles again with their offsets.
template <class T>
__global__ __launch_bounds__(RS_THREADS) void scan_reduce_kernel(const T *__restrict__ x,
                                                                 int64_t n,
                                                                 T *__restrict__ sums) {
    __shared__ int64_t s_tmp[RS_THREADS / WAVE];
    const int64_t base = int64_t(blockIdx.x) * RS_TILE;
    int64_t v = 0;
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const int64_t idx = base + int64_t(j) * RS_THREADS + threadIdx.x;
        if (idx < n) v += x[idx];
    }
    int64_t tot;
    block_exclusive_scan(v, s_tmp, tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = T(tot);
}

template <class T>
__global__ __launch_bounds__(1024) void scan_top_kernel(T *__restrict__ sums, int64_t m) {
    __shared__ int64_t s_tmp[1024 / WAVE];
    int64_t carry = 0;
    for (int64_t base = 0; base < m; base += 1024) {
        const int64_t idx = base + threadIdx.x;
        const int64_t v = idx < m ? sums[idx] : 0;
        int64_t tot;
        const int64_t ex = block_exclusive_scan(v, s_tmp, tot);
        if (idx < m) sums[idx] = T(carry + ex);
        carry += tot;
    }
}

template <class T>
__global__ __launch_bounds__(RS_THREADS) void scan_down_kernel(T *__restrict__ x, int64_t n,
                                                               const T *__restrict__ sums) {
    __shared__ int64_t s_tmp[RS_THREADS / WAVE];
    __shared__ T s_x[RS_TILE];
    // coalesced loads into LDS; thread t then owns elements
    // [RS_ITEMS t, RS_ITEMS (t+1)) of the tile
    const int64_t base = int64_t(blockIdx.x) * RS_TILE;
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const int q = j * RS_THREADS + threadIdx.x;
        s_x[q] = base + q < n ? x[base + q] : T(0);
    }
    __syncthreads();
    T v[RS_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        v[j] = s_x[threadIdx.x * RS_ITEMS + j];
        s += v[j];
    }
    int64_t tot;
    int64_t run = block_exclusive_scan(s, s_tmp, tot) + sums[blockIdx.x];
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        s_x[threadIdx.x * RS_ITEMS + j] = T(run);
        run += v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const int q = j * RS_THREADS + threadIdx.x;
        if (base + q < n) x[base + q] = s_x[q];
    }
}

// One stable radix pass.  Wave w of a tile ranks its RS_ITEMS * 64 elements in
// order (lanes with equal digits found by eight ballots), the tile's elements
// are placed in LDS sorted by digit, and each digit's run is written out
// contiguously at its scanned offset.
__global__ __launch_bounds__(RS_THREADS) void rs_scatter_kernel(
    const uint64_t *__restrict__ kin, const int32_t *__restrict__ vin, int64_t n, int shift,
    const uint32_t *__restrict__ goff, int64_t ntiles, uint64_t *__restrict__ kout,
    int32_t *__restrict__ vout) {
    constexpr int WAVES = RS_THREADS / WAVE;
    __shared__ uint64_t s_key[RS_TILE];
    __shared__ int32_t s_val[RS_TILE];
    __shared__ uint32_t s_wrun[WAVES][256];  // per wave: elements of each digit so far
    __shared__ uint32_t s_start[256];        // first LDS slot of each digit
    __shared__ uint32_t s_glob[256];         // global offset of each digit's run
    const int t = threadIdx.x, w = t / WAVE, l = lane();
    for (int q = t; q < WAVES * 256; q += RS_THREADS) (&s_wrun[0][0])[q] = 0;
    s_glob[t] = goff[int64_t(t) * ntiles + blockIdx.x];
    __syncthreads();
    // wave w takes elements [base + 64 RS_ITEMS w, base + 64 RS_ITEMS (w+1)), 64 per step
    const int64_t wbase = int64_t(blockIdx.x) * RS_TILE + int64_t(w) * WAVE * RS_ITEMS;
    uint64_t k[RS_ITEMS];
    int32_t v[RS_ITEMS];
    uint32_t d[RS_ITEMS], r[RS_ITEMS];
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const int64_t idx = wbase + int64_t(j) * WAVE + l;
        k[j] = idx < n ? kin[idx] : 0;
        v[j] = idx < n ? vin[idx] : 0;
    }
    const uint64_t lt = (1ull << l) - 1;
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const int64_t idx = wbase + int64_t(j) * WAVE + l;
        const bool act = idx < n;
        d[j] = uint32_t(k[j] >> shift) & 255u;
        uint64_t peers = __ballot(act);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (d[j] >> bit) & 1u;
            const uint64_t m = __ballot(on);
            peers &= on ? m : ~m;
        }
        r[j] = 0;
        if (act) {
            r[j] = s_wrun[w][d[j]] + __popcll(peers & lt);
            // the highest lane of each digit group advances the wave's count
            if ((peers >> l) == 1ull) s_wrun[w][d[j]] += __popcll(peers);
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    {
        // digit t: its first LDS slot, and each wave's start inside its run
        uint32_t cnt = 0;
        for (int q = 0; q < WAVES; ++q) {
            const uint32_t c = s_wrun[q][t];
            s_wrun[q][t] = cnt;  // now: offset of wave q's elements within digit t's run
            cnt += c;
        }
        // exclusive scan of the digit totals over the block (256 digits, 256 threads)
        __shared__ int64_t s_tmp[RS_THREADS / WAVE];
        int64_t tot;
        s_start[t] = uint32_t(block_exclusive_scan(int64_t(cnt), s_tmp, tot));
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RS_ITEMS; ++j) {
        const int64_t idx = wbase + int64_t(j) * WAVE + l;
        if (idx < n) {
            const uint32_t pos = s_start[d[j]] + s_wrun[w][d[j]] + r[j];
            s_key[pos] = k[j];
            s_val[pos] = v[j];
        }
    }
    __syncthreads();
    const int64_t tbase = int64_t(blockIdx.x) * RS_TILE;
    const int64_t cnt = imin(RS_TILE, n - tbase);
    for (int64_t q = t; q < cnt; q += RS_THREADS) {
        const uint64_t key = s_key[q];
        const uint32_t dg = uint32_t(key >> shift) & 255u;
        const int64_t dst = int64_t(s_glob[dg]) + (q - s_start[dg]);
        if (dst < n) {
            kout[dst] = key;
            vout[dst] = s_val[q];
        }
    }
}

// flags[p] = 1 where the sorted key changes (p = 0 included).
__global__ __launch_bounds__(RS_THREADS) void sa_heads_kernel(const uint64_t *__restrict__ keys,
                                                              int64_t n,
                                                              uint32_t *__restrict__ flags) {
    const int64_t p = int64_t(blockIdx.x) * RS_THREADS + threadIdx.x;
    if (p < n) flags[p] = p == 0 || keys[p] != keys[p - 1] ? 1u : 0u;
}

// After a sort of the m active suffixes (vals, by key): group j's members
// are the runs of equal keys.  E = exclusive scan of the run-start flags,
// so E[j] + flag[j] - 1 is the run index of j; first[g] = index of run g's
// first element (first[runs] = m).
__global__ __launch_bounds__(RS_THREADS) void sa_first_kernel(const uint64_t *__restrict__ keys,
                                                              const uint32_t *__restrict__ E,
                                                              int64_t m,
                                                              uint32_t *__restrict__ first) {
    const int64_t j = int64_t(blockIdx.x) * RS_THREADS + threadIdx.x;
    if (j >= m) return;
    const uint32_t f = j == 0 || keys[j] != keys[j - 1] ? 1u : 0u;
    if (f) first[E[j]] = uint32_t(j);
    if (j == m - 1) first[E[j] + f] = uint32_t(m);
}

// Rank of every sorted active suffix = position (in the full sorted order)
// of its run's first element; suffixes in runs of one are final.  Writes the
// suffix into its place in the full order, and active[j] = run size >= 2.
// pos == nullptr: the m elements are the full order itself.
__global__ __launch_bounds__(RS_THREADS) void sa_rank_kernel(
    const uint64_t *__restrict__ keys, const uint32_t *__restrict__ E,
    const uint32_t *__restrict__ first, int64_t m, const int32_t *__restrict__ vals,
    const uint32_t *__restrict__ pos, int64_t n, uint32_t *__restrict__ rank,
    int32_t *__restrict__ order, uint32_t *__restrict__ active) {
    const int64_t j = int64_t(blockIdx.x) * RS_THREADS + threadIdx.x;
    if (j >= m) return;
    const uint32_t f = j == 0 || keys[j] != keys[j - 1] ? 1u : 0u;
    const uint32_t g = E[j] + f - 1u;
    const uint32_t h0 = first[g], h1 = first[g + 1];
    const uint32_t at = pos ? pos[j] : uint32_t(j);
    const uint32_t head = pos ? pos[h0] : h0;
    const int64_t i = vals[j];
    if (i >= 0 && i < n) rank[i] = head;
    if (at < uint64_t(n)) order[at] = int32_t(i);
    active[j] = h1 - h0 >= 2u ? 1u : 0u;
}

// Keep the active elements: their places in the full order and their
// suffixes, in sorted order (A = exclusive scan of the active flags).
__global__ __launch_bounds__(RS_THREADS) void sa_compact_kernel(
    const uint64_t *__restrict__ keys, const uint32_t *__restrict__ E,
    const uint32_t *__restrict__ first, const uint32_t *__restrict__ A, int64_t m,
    const int32_t *__restrict__ vals, const uint32_t *__restrict__ pos,
    uint32_t *__restrict__ pos_out, int32_t *__restrict__ vals_out,
    uint32_t *__restrict__ gid_out, uint32_t *count) {
    const int64_t j = int64_t(blockIdx.x) * RS_THREADS + threadIdx.x;
    if (j >= m) return;
    const uint32_t f = j == 0 || keys[j] != keys[j - 1] ? 1u : 0u;
    const uint32_t g = E[j] + f - 1u;
    const bool act = first[g + 1] - first[g] >= 2u;
    if (act) {
        pos_out[A[j]] = pos ? pos[j] : uint32_t(j);
        vals_out[A[j]] = vals[j];
        gid_out[A[j]] = g;  // run index: orders the runs like their ranks
    }
    if (j == m - 1) *count = A[j] + (act ? 1u : 0u);
}

// Doubling keys of the active suffixes: (run index of suffix i -- ordered as
// the ranks of the runs --, 1 + rank of suffix i + h, or 0 past the end of
// i's string).  A key is below runs (n + 1), so early rounds with few runs
// sort fewer bits.
__global__ __launch_bounds__(RS_THREADS) void sa_keys_kernel(
    const int32_t *__restrict__ vals, const uint32_t *__restrict__ gid, int64_t m,
    const uint32_t *__restrict__ rank, int64_t n, Segs segs, int64_t h,
    uint64_t *__restrict__ keys) {
    const int64_t j = int64_t(blockIdx.x) * RS_THREADS + threadIdx.x;
    if (j >= m) return;
    const int64_t i = vals[j];
    uint64_t r2 = 0;
    if (i >= 0 && i < n) {
        const int64_t e = segs.end(segs.find(i));
        if (i + h < e) r2 = uint64_t(rank[i + h]) + 1;
    }
    keys[j] = uint64_t(gid[j]) * uint64_t(n + 1) + r2;
}

// The result: segment-local suffix starts in sorted order.
__global__ __launch_bounds__(RS_THREADS) void sa_out_kernel(const int32_t *__restrict__ vals,
                                                            int64_t n, Segs segs,
                                                            int32_t *__restrict__ sa) {
    __shared__ int32_t s_b;
    const int64_t p0 = int64_t(blockIdx.x) * RS_THREADS;
    int32_t b = block_segment(segs, imin(p0, n - 1), &s_b);
    const int64_t p = p0 + threadIdx.x;
    if (p >= n) return;
    b = segs.advance(b, p);
    sa[p] = int32_t(int64_t(vals[p]) - segs.begin(b));
}

struct SaWork {
    uint64_t *key[2];
    int32_t *val[2];
    int32_t *order;          // the full sorted order of suffixes
    uint32_t *pos[2];        // active elements' places in the full order
    uint32_t *rank, *aux, *act, *first, *gid, *hist, *sums, *mask, *count;
    int64_t ntiles, hist_tiles;
    size_t bytes;
};

SaWork sa_layout(void *base, int64_t n) {
    SaWork w{};
    size_t at = 0;
    auto take = [&](size_t bytes) { size_t o = at; at = align256(at + bytes); return o; };
    const int64_t nn = n > 0 ? n : 1;
    w.ntiles = (nn + RS_TILE - 1) / RS_TILE;
    w.hist_tiles = (256 * w.ntiles + RS_TILE - 1) / RS_TILE;
    const size_t k0 = take(size_t(nn) * 8), k1 = take(size_t(nn) * 8);
    const size_t v0 = take(size_t(nn) * 4), v1 = take(size_t(nn) * 4);
    const size_t rk = take(size_t(nn) * 4), ax = take(size_t(nn) * 4);
    const size_t od = take(size_t(nn) * 4), p0 = take(size_t(nn) * 4), p1 = take(size_t(nn) * 4);
    const size_t ac = take(size_t(nn) * 4), fi = take(size_t(nn + 1) * 4);
    const size_t gd = take(size_t(nn) * 4);
    const size_t hs = take(size_t(256 * w.ntiles) * 4);
    const int64_t sum_n = w.ntiles > w.hist_tiles ? w.ntiles : w.hist_tiles;
    const size_t sm = take(size_t(sum_n) * 4);
    const size_t mk = take(32), ct = take(8);
    w.bytes = at;
    if (base) {
        char *b = static_cast<char *>(base);
        w.key[0] = reinterpret_cast<uint64_t *>(b + k0);
        w.key[1] = reinterpret_cast<uint64_t *>(b + k1);
        w.val[0] = reinterpret_cast<int32_t *>(b + v0);
        w.val[1] = reinterpret_cast<int32_t *>(b + v1);
        w.rank = reinterpret_cast<uint32_t *>(b + rk);
        w.aux = reinterpret_cast<uint32_t *>(b + ax);
        w.order = reinterpret_cast<int32_t *>(b + od);
        w.pos[0] = reinterpret_cast<uint32_t *>(b + p0);
        w.pos[1] = reinterpret_cast<uint32_t *>(b + p1);
        w.act = reinterpret_cast<uint32_t *>(b + ac);
        w.first = reinterpret_cast<uint32_t *>(b + fi);
        w.gid = reinterpret_cast<uint32_t *>(b + gd);
        w.count = reinterpret_cast<uint32_t *>(b + ct);
        w.hist = reinterpret_cast<uint32_t *>(b + hs);
        w.sums = reinterpret_cast<uint32_t *>(b + sm);
        w.mask = reinterpret_cast<uint32_t *>(b + mk);
    }
    return w;
}

template <class T>
int run_scan(T *x, int64_t n, T *sums, hipStream_t st) {
    const int64_t tiles = (n + RS_TILE - 1) / RS_TILE;
    LAUNCH(scan_reduce_kernel<T>, dim3(unsigned(tiles)), dim3(RS_THREADS), 0, st, x, n, sums);
    LAUNCH(scan_top_kernel<T>, dim3(1), dim3(1024), 0, st, sums, tiles);
    LAUNCH(scan_down_kernel<T>, dim3(unsigned(tiles)), dim3(RS_THREADS), 0, st, x, n, sums);
    return check_launch("scan kernels");
}

// Sorts (key, val) pairs in w.key[cur] / w.val[cur] by key bits [lo, hi);
// returns the buffer index holding the result.
int radix_sort(SaWork &w, int64_t n, int lo, int hi, int cur, hipStream_t st, int *out_cur) {
    for (int shift = lo; shift < hi; shift += 8) {
        LAUNCH(rs_hist_kernel, dim3(unsigned(w.ntiles)), dim3(RS_THREADS), 0, st, w.key[cur], n,
               shift, w.hist, w.ntiles);
        int rc = run_scan(w.hist, 256 * w.ntiles, w.sums, st);
        if (rc) return rc;
        LAUNCH(rs_scatter_kernel, dim3(unsigned(w.ntiles)), dim3(RS_THREADS), 0, st, w.key[cur],
               w.val[cur], n, shift, w.hist, w.ntiles, w.key[cur ^ 1], w.val[cur ^ 1]);
        if ((rc = check_launch("rs_scatter_kernel"))) return rc;
        cur ^= 1;
    }
    *out_cur = cur;
    return LRQ_OK;
}

int bits_for(uint64_t v) {  // bits needed to hold v
    int b = 0;
    while (b < 64 && (v >> b) != 0) ++b;
    return b;
}


// ============================================================================
// Raw LLR walks (Section 4.1; Algorithms 1 and 3): the leftmost LR, or all
// LRs, of every position straight from the raw LLR array L, without the
// compaction.  Within a string i + L_i never decreases (an LLR at i of length
// L minus its first character is a repeat at i + 1, so L_{i+1} >= L_i - 1),
// hence the LLRs covering k are exactly i in [lo(k), k]: walking left from k
// the walk stops at the first i whose LLR ends before k.  O(alpha) work per
// position, alpha = mean L (Lemma 4), against O(beta) for the compact scans;
// a walk longer than max_walk stops and sets LRQ_ERR_WALK (its position's
// answer is then incomplete), so that long-repeat texts cannot run away.
// ============================================================================

enum RawMode { RAW_LEFTMOST = 0, RAW_COUNT = 1, RAW_EMIT = 2 };

// Lemma 1: L_i = max(PLCP[i], NLCP[i]).
__global__ __launch_bounds__(256) void llr_lengths_kernel(const int4 *__restrict__ pn4,
                                                          int64_t total,
                                                          int2 *__restrict__ L2,
                                                          int32_t *__restrict__ L) {
    const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;  // pair index
    const int64_t p0 = 2 * q;
    if (p0 + 1 < total) {
        const int4 v = pn4[q];
        L2[q] = make_int2(v.x > v.y ? v.x : v.y, v.z > v.w ? v.z : v.w);
    } else if (p0 < total) {
        const int2 v = reinterpret_cast<const int2 *>(pn4)[p0];
        L[p0] = v.x > v.y ? v.x : v.y;
    }
}

template <int MODE>
__global__ __launch_bounds__(256) void lr_raw_kernel(const int32_t *__restrict__ L, int64_t total,
                                                     Segs segs, int32_t max_walk,
                                                     int2 *__restrict__ out,
                                                     int64_t *__restrict__ offsets,
                                                     int2 *__restrict__ recs, int64_t capacity,
                                                     uint32_t *err) {
    __shared__ int32_t s_b;
    const int64_t k0 = int64_t(blockIdx.x) * blockDim.x;
    int32_t b = segs.off ? block_segment(segs, k0, &s_b) : 0;
    const int64_t k = k0 + threadIdx.x;
    if (k >= total) return;
    b = segs.advance(b, k);
    const int64_t sb = segs.begin(b), se = segs.end(b);
    // walk left: the longest covering LLR (ties: the smallest start) and the
    // number of covering LLRs of that length
    int32_t best = 0, cnt = 0;
    int64_t bs = -1, lo = k + 1;
    int32_t steps = 0;
    bool bad = false;
    for (int64_t i = k; i >= sb; --i) {
        const int32_t li = L[i];
        if (i + li - 1 < k) break;  // this LLR ends before k, and so do all before it
        if (i + li > se) {          // an LLR cannot run past its string
            bad = true;
            break;
        }
        if (++steps > max_walk) {
            raise_err(err, LRQ_ERR_WALK);
            break;
        }
        lo = i;
        if (li > best) {
            best = li;
            bs = i;
            cnt = 1;
        } else if (li == best) {
            bs = i;
            ++cnt;
        }
    }
    if (bad) raise_err(err, LRQ_ERR_SA);
    if (MODE == RAW_LEFTMOST || (MODE == RAW_COUNT && out))
        out[k] = bs >= 0 ? make_int2(int32_t(bs - sb), best) : make_int2(-1, 0);
    if (MODE == RAW_COUNT) {
        offsets[k] = cnt;  // scanned into offsets afterwards
    } else if (MODE == RAW_EMIT) {
        int64_t w = offsets[k];
        if (best > 0) {
            for (int64_t i = lo; i <= k; ++i) {
                const int32_t li = L[i];
                if (li != best) continue;
                if (w < capacity) recs[w] = make_int2(int32_t(i - sb), best);
                else raise_err(err, LRQ_ERR_CAPACITY);
                ++w;
            }
        }
    }
}

}  // namespace
}  // namespace lrq

extern "C" {

int lrq_sa_work_bytes(int64_t total, int32_t nseg, size_t *bytes) {
    clear_error();
    if (!bytes) { set_error("bytes is NULL"); return LRQ_EINVAL; }
    if (total < 0 || nseg < 1) { set_error("total < 0 or nseg < 1"); return LRQ_EINVAL; }
    if (total > LRQ_MAX_TOTAL) { set_error("total > LRQ_MAX_TOTAL"); return LRQ_ERANGE; }
    *bytes = sa_layout(nullptr, total).bytes;
    return LRQ_OK;
}

int lrq_build_sa(const uint8_t *d_text, int64_t total, const int64_t *d_seg_off, int32_t nseg,
                 int32_t *d_sa, void *d_work, size_t work_bytes, void *stream) {
    clear_error();
    if (total < 0 || nseg < 1) { set_error("total < 0 or nseg < 1"); return LRQ_EINVAL; }
    if (total > LRQ_MAX_TOTAL) { set_error("total > LRQ_MAX_TOTAL"); return LRQ_ERANGE; }
    if (!d_seg_off && nseg != 1) { set_error("seg_off is NULL but nseg != 1"); return LRQ_EINVAL; }
    if (total == 0) return LRQ_OK;
    if (!d_text || !d_sa || !d_work) { set_error("d_text / d_sa / d_work is NULL"); return LRQ_EINVAL; }
    if (misaligned(d_text, 8)) { set_error("d_text not 8-byte aligned"); return LRQ_EINVAL; }
    if (misaligned(d_work, 256)) { set_error("d_work not 256-byte aligned"); return LRQ_EINVAL; }
    SaWork w = sa_layout(d_work, total);
    if (work_bytes < w.bytes) {
        set_error("work has %zu bytes, needs %zu", work_bytes, w.bytes);
        return LRQ_ENOMEM;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Segs segs{d_seg_off, nseg, total};
    const int64_t n = total;
    const unsigned grid = grid_for(n, RS_THREADS);
    int rc;
    // the byte values present, then the code width and characters per key
    if ((rc = run_zero(reinterpret_cast<uint64_t *>(w.mask), 4, st))) return rc;
    {
        const int64_t words = n >> 3;
        int64_t gb = (words + 4 * 1024 - 1) / (4 * 1024);
        gb = gb < 1 ? 1 : (gb > 256 ? 256 : gb);
        LAUNCH(alpha_kernel, dim3(unsigned(gb)), dim3(1024), 0, st, d_text, n, w.mask);
        if ((rc = check_launch("alpha_kernel"))) return rc;
    }
    uint32_t mask[8];
    if (hipMemcpyAsync(mask, w.mask, sizeof mask, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        set_error("reading the byte-value mask: %s", hipGetErrorString(hipGetLastError()));
        return LRQ_EDEVICE;
    }
    int sigma = 0;
    for (int q = 0; q < 8; ++q) sigma += __builtin_popcount(mask[q]);
    const int cb = bits_for(uint64_t(sigma));  // codes 1..sigma, 0 past the end
    const int sbits = nseg > 1 ? bits_for(uint64_t(nseg - 1)) : 0;
    const int K = (64 - sbits) / cb;
    LAUNCH(sa_key0_kernel, dim3(grid), dim3(RS_THREADS), 0, st, d_text, n, segs, w.mask, cb, K,
           sbits, w.key[0], w.val[0]);
    if ((rc = check_launch("sa_key0_kernel"))) return rc;
    int cur = 0;
    const int lo = ((64 - sbits - cb * K) / 8) * 8;
    if ((rc = radix_sort(w, n, lo, 64, cur, st, &cur))) return rc;
    // Refinement (Larsson and Sadakane's scheme over the doubling): every
    // round sorts only the suffixes whose group (equal keys so far) has two
    // or more members; the rank of a suffix is the position of its group's
    // first element in the full order, final once its group is a singleton.
    int64_t m = n;             // active elements, sorted, in key[cur] / val[cur]
    const uint32_t *pos = nullptr;  // their places in the full order (round 0: all)
    int pc = 0;
    int64_t h = K;
    for (int round = 0;; ++round) {
        const unsigned gm = grid_for(m, RS_THREADS);
        LAUNCH(sa_heads_kernel, dim3(gm), dim3(RS_THREADS), 0, st, w.key[cur], m, w.aux);
        if ((rc = run_scan(w.aux, m, w.sums, st))) return rc;
        LAUNCH(sa_first_kernel, dim3(gm), dim3(RS_THREADS), 0, st, w.key[cur], w.aux, m, w.first);
        LAUNCH(sa_rank_kernel, dim3(gm), dim3(RS_THREADS), 0, st, w.key[cur], w.aux, w.first, m,
               w.val[cur], pos, n, w.rank, w.order, w.act);
        if ((rc = run_scan(w.act, m, w.sums, st))) return rc;
        LAUNCH(sa_compact_kernel, dim3(gm), dim3(RS_THREADS), 0, st, w.key[cur], w.aux, w.first,
               w.act, m, w.val[cur], pos, w.pos[pc], w.val[cur ^ 1], w.gid, w.count);
        if ((rc = check_launch("suffix ranks"))) return rc;
        uint32_t left = 0, runs = 0;
        if (hipMemcpyAsync(&left, w.count, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(&runs, w.aux + (m - 1), 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            set_error("reading the active count: %s", hipGetErrorString(hipGetLastError()));
            return LRQ_EDEVICE;
        }
        runs += 1;  // E[m-1] + (a flag of at most 1) bounds the run indices
        if (left == 0) break;
        if (h >= n || round > 64) {  // cannot happen: suffixes of one string differ in length
            set_error("suffix ranks did not separate after %d rounds", round);
            return LRQ_EDATA;
        }
        m = left;
        pos = w.pos[pc];
        pc ^= 1;
        cur ^= 1;
        LAUNCH(sa_keys_kernel, dim3(grid_for(m, RS_THREADS)), dim3(RS_THREADS), 0, st, w.val[cur],
               w.gid, m, w.rank, n, segs, h, w.key[cur]);
        if ((rc = check_launch("sa_keys_kernel"))) return rc;
        const int kb = bits_for(uint64_t(runs) * uint64_t(n + 1) + uint64_t(n));
        if ((rc = radix_sort(w, m, 0, kb, cur, st, &cur))) return rc;
        // the sort moved the pairs; the positions stay with their slots, so
        // the sorted element j of the round goes to place pos[j]
        h *= 2;
    }
    LAUNCH(sa_out_kernel, dim3(grid), dim3(RS_THREADS), 0, st, w.order, n, segs, d_sa);
    return check_launch("sa_out_kernel");
}


int lrq_llr_lengths(const int32_t *d_pn, int64_t total, int32_t *d_L, void *stream) {
    clear_error();
    if (total < 0) { set_error("total < 0"); return LRQ_EINVAL; }
    if (total > LRQ_MAX_TOTAL) { set_error("total > LRQ_MAX_TOTAL"); return LRQ_ERANGE; }
    if (total == 0) return LRQ_OK;
    if (!d_pn || !d_L) { set_error("d_pn / d_L is NULL"); return LRQ_EINVAL; }
    if (misaligned(d_pn, 16) || misaligned(d_L, 8)) { set_error("d_pn not 16-byte or d_L not 8-byte aligned"); return LRQ_EINVAL; }
    hipStream_t st = static_cast<hipStream_t>(stream);
    LAUNCH(llr_lengths_kernel, dim3(grid_for((total + 1) / 2, 256)), dim3(256), 0, st,
           reinterpret_cast<const int4 *>(d_pn), total, reinterpret_cast<int2 *>(d_L), d_L);
    return check_launch("llr_lengths_kernel");
}

static int32_t raw_walk_bound(int32_t max_walk) { return max_walk > 0 ? max_walk : 65536; }

int lrq_lr_leftmost_raw(const int32_t *d_L, int64_t total, const int64_t *d_seg_off, int32_t nseg,
                        int32_t max_walk, lrq_rec *d_out, void *d_scratch, size_t scratch_bytes,
                        void *stream) {
    clear_error();
    int rc = check_common(total, d_seg_off, nseg, d_scratch, scratch_bytes);
    if (rc) return rc;
    if (total == 0) return LRQ_OK;
    if (!d_L || !d_out || misaligned(d_out, 8)) { set_error("d_L / d_out NULL or d_out not 8-byte aligned"); return LRQ_EINVAL; }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Segs segs{d_seg_off, nseg, total};
    LAUNCH(lr_raw_kernel<RAW_LEFTMOST>, dim3(grid_for(total, 256)), dim3(256), 0, st, d_L, total,
           segs, raw_walk_bound(max_walk), reinterpret_cast<int2 *>(d_out), nullptr, nullptr,
           int64_t(0), at<uint32_t>(d_scratch, HDR_ERR));
    return check_launch("lr_raw_kernel");
}

int lrq_lr_all_raw(const int32_t *d_L, int64_t total, const int64_t *d_seg_off, int32_t nseg,
                   int32_t max_walk, lrq_rec *d_out, int64_t *d_offsets, lrq_rec *d_recs,
                   int64_t capacity, int64_t *h_total, void *d_scratch, size_t scratch_bytes,
                   void *stream) {
    clear_error();
    int rc = check_common(total, d_seg_off, nseg, d_scratch, scratch_bytes);
    if (rc) return rc;
    if (!d_offsets || misaligned(d_offsets, 8)) { set_error("d_offsets NULL or not 8-byte aligned"); return LRQ_EINVAL; }
    if (capacity < 0 || (capacity > 0 && (!d_recs || misaligned(d_recs, 8)))) { set_error("bad d_recs / capacity"); return LRQ_EINVAL; }
    if (total > 0 && !d_L) { set_error("d_L is NULL"); return LRQ_EINVAL; }
    if (d_out && misaligned(d_out, 8)) { set_error("d_out not 8-byte aligned"); return LRQ_EINVAL; }
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (total == 0) {
        if ((rc = run_zero(reinterpret_cast<uint64_t *>(d_offsets), 1, st))) return rc;
        if (h_total) *h_total = 0;
        return LRQ_OK;
    }
    const Segs segs{d_seg_off, nseg, total};
    const Layout L = layout(total, nseg);
    const int32_t mw = raw_walk_bound(max_walk);
    uint32_t *err = at<uint32_t>(d_scratch, HDR_ERR);
    // counts into offsets[0, total), offsets[total] = 0, then one exclusive
    // scan over total + 1 entries gives the CSR offsets and the record total
    if ((rc = run_zero(reinterpret_cast<uint64_t *>(d_offsets + total), 1, st))) return rc;
    LAUNCH(lr_raw_kernel<RAW_COUNT>, dim3(grid_for(total, 256)), dim3(256), 0, st, d_L, total,
           segs, mw, reinterpret_cast<int2 *>(d_out), d_offsets, nullptr, int64_t(0), err);
    if ((rc = check_launch("lr_raw_kernel"))) return rc;
    // the scan's tile sums (one per 4096 entries) use the LR scans' state words
    if ((rc = run_scan(d_offsets, total + 1, at<int64_t>(d_scratch, L.lr_state), st))) return rc;
    LAUNCH(lr_raw_kernel<RAW_EMIT>, dim3(grid_for(total, 256)), dim3(256), 0, st, d_L, total,
           segs, mw, nullptr, d_offsets, reinterpret_cast<int2 *>(d_recs), capacity, err);
    if ((rc = check_launch("lr_raw_kernel"))) return rc;
    if (!h_total) return LRQ_OK;
    hipError_t e = hipMemcpyAsync(h_total, d_offsets + total, sizeof(int64_t),
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) { set_error("reading the record total: %s", hipGetErrorString(e)); return LRQ_EDEVICE; }
    if (*h_total > capacity) {
        set_error("%lld records, capacity %lld", (long long)*h_total, (long long)capacity);
        return LRQ_ENOSPC;
    }
    return LRQ_OK;
}

}  // extern "C"

namespace lrq {
namespace {

// Point queries in either mode.  Leftmost: one launch.  All: counts (and,
// with d_out, the leftmost records) into d_offsets[0, m), d_offsets[m] = 0,
// one exclusive scan over m + 1 entries, then the records.  err is the error
// word; sums holds the scan's tile sums, ceil((m + 1) / RS_TILE) words
// (written before they are read, so they need no clearing).
template <class SRC>
int query_run(const SRC &src, const typename SRC::Pos *d_pos, int64_t m, int32_t mode,
              void *d_out, int64_t *d_offsets, void *d_recs, int64_t capacity, int64_t *h_total,
              uint32_t *err, int64_t *sums, hipStream_t st) {
    using E = typename SRC::E;
    E *out = reinterpret_cast<E *>(d_out);
    int rc;
    if (mode == LRQ_LEFTMOST) {
        if (m == 0) return LRQ_OK;
        LAUNCH(query_kernel<QUERY_LEFTMOST>, dim3(grid_for(m, 256)), dim3(256), 0, st, src, d_pos,
               m, out, nullptr, nullptr, int64_t(0), err);
        return check_launch("query_kernel");
    }
    if ((rc = run_zero(reinterpret_cast<uint64_t *>(d_offsets + m), 1, st))) return rc;
    if (m > 0) {
        LAUNCH(query_kernel<QUERY_COUNT>, dim3(grid_for(m, 256)), dim3(256), 0, st, src, d_pos, m,
               out, d_offsets, nullptr, int64_t(0), err);
        if ((rc = check_launch("query_kernel"))) return rc;
        if ((rc = run_scan(d_offsets, m + 1, sums, st))) return rc;
        LAUNCH(query_kernel<QUERY_EMIT>, dim3(grid_for(m, 256)), dim3(256), 0, st, src, d_pos, m,
               nullptr, d_offsets, reinterpret_cast<E *>(d_recs), capacity, err);
        if ((rc = check_launch("query_kernel"))) return rc;
    }
    if (!h_total) return LRQ_OK;
    if ((rc = read_total(h_total, d_offsets + m, st))) return rc;
    if (*h_total > capacity) {
        set_error("%lld records, capacity %lld", (long long)*h_total, (long long)capacity);
        return LRQ_ENOSPC;
    }
    return LRQ_OK;
}

// The all-mode scan's tile sums inside a caller's scratch buffer: the LR
// scans' state words of a layout for m positions, at least
// ceil((m + 1) / RS_TILE) words (lr_tile <= RS_TILE).
int64_t *query_sums(void *d_scratch, int64_t m) {
    static_assert(RS_TILE >= 4096, "one LR-state word per scan tile at the largest lr_tile");
    return at<int64_t>(d_scratch, layout(m, 1).lr_state);
}

// Argument checks shared by both point-query calls.
int check_query(int64_t n_scratch, const void *d_pos, int64_t m, int32_t mode,
                const void *d_out, const int64_t *d_offsets, const void *d_recs,
                int64_t capacity, void *d_scratch, size_t scratch_bytes,
                int64_t max_total = LRQ_MAX_TOTAL) {
    if (m < 0) { set_error("m < 0"); return LRQ_EINVAL; }
    if (m > max_total) { set_error("m = %lld queries, beyond the size limit", (long long)m); return LRQ_ERANGE; }
    if (mode != LRQ_LEFTMOST && mode != LRQ_ALL) { set_error("mode %d", mode); return LRQ_EINVAL; }
    // all mode scans m + 1 counts with the scratch's state words
    int rc = check_common(mode == LRQ_ALL && m > n_scratch ? m : n_scratch, nullptr, 1, d_scratch,
                          scratch_bytes, max_total);
    if (rc) return rc;
    if (m > 0 && !d_pos) { set_error("d_pos is NULL"); return LRQ_EINVAL; }
    if (mode == LRQ_LEFTMOST) {
        if (m > 0 && (!d_out || misaligned(d_out, 8))) { set_error("d_out NULL or not 8-byte aligned"); return LRQ_EINVAL; }
        return LRQ_OK;
    }
    if (!d_offsets || misaligned(d_offsets, 8)) { set_error("d_offsets NULL or not 8-byte aligned"); return LRQ_EINVAL; }
    if (capacity < 0 || (capacity > 0 && (!d_recs || misaligned(d_recs, 8)))) { set_error("bad d_recs / capacity"); return LRQ_EINVAL; }
    if (d_out && misaligned(d_out, 8)) { set_error("d_out not 8-byte aligned"); return LRQ_EINVAL; }
    return LRQ_OK;
}

}  // namespace
}  // namespace lrq

extern "C" {

int lrq_query_positions(const lrq_rec *d_llrc, const int64_t *d_llrc_blocks, int64_t n,
                        const int32_t *d_pos, int64_t m, int32_t mode, lrq_rec *d_out,
                        int64_t *d_offsets, lrq_rec *d_recs, int64_t capacity, int64_t *h_total,
                        void *d_scratch, size_t scratch_bytes, void *stream) {
    clear_error();
    int rc = check_query(n, d_pos, m, mode, d_out, d_offsets, d_recs, capacity, d_scratch,
                         scratch_bytes);
    if (rc) return rc;
    if (m > 0 && (rc = check_index(d_llrc, d_llrc_blocks))) return rc;
    const OneString<int32_t> src{reinterpret_cast<const int2 *>(d_llrc), d_llrc_blocks, n};
    return query_run(src, d_pos, m, mode, d_out, d_offsets, d_recs, capacity, h_total,
                     at<uint32_t>(d_scratch, HDR_ERR), query_sums(d_scratch, m),
                     static_cast<hipStream_t>(stream));
}

int lrq_query_multi(const lrq_string_ref *d_refs, int32_t nrefs, const int32_t *d_sid,
                    const int32_t *d_pos, int64_t m, int32_t mode, lrq_rec *d_out,
                    int64_t *d_offsets, lrq_rec *d_recs, int64_t capacity, int64_t *h_total,
                    void *d_scratch, size_t scratch_bytes, void *stream) {
    clear_error();
    int rc = check_query(0, d_pos, m, mode, d_out, d_offsets, d_recs, capacity, d_scratch,
                         scratch_bytes);
    if (rc) return rc;
    if (nrefs < 0) { set_error("nrefs < 0"); return LRQ_EINVAL; }
    if (m > 0 && (!d_refs || !d_sid)) { set_error("d_refs / d_sid is NULL"); return LRQ_EINVAL; }
    if (m > 0 && misaligned(d_refs, 8)) { set_error("d_refs not 8-byte aligned"); return LRQ_EINVAL; }
    const ManyStrings src{d_refs, nrefs, d_sid};
    return query_run(src, d_pos, m, mode, d_out, d_offsets, d_recs, capacity, h_total,
                     at<uint32_t>(d_scratch, HDR_ERR), query_sums(d_scratch, m),
                     static_cast<hipStream_t>(stream));
}

int lrq64_query_positions(const lrq_rec64 *d_llrc, const int64_t *d_llrc_blocks, int64_t n,
                          const int64_t *d_pos, int64_t m, int32_t mode, lrq_rec64 *d_out,
                          int64_t *d_offsets, lrq_rec64 *d_recs, int64_t capacity,
                          int64_t *h_total, void *d_scratch, size_t scratch_bytes, void *stream) {
    clear_error();
    int rc = check_query(n, d_pos, m, mode, d_out, d_offsets, d_recs, capacity, d_scratch,
                         scratch_bytes, LRQ64_MAX_TOTAL);
    if (rc) return rc;
    if (d_out && misaligned(d_out, 16)) { set_error("d_out not 16-byte aligned"); return LRQ_EINVAL; }
    if (mode == LRQ_ALL && capacity > 0 && misaligned(d_recs, 16)) { set_error("d_recs not 16-byte aligned"); return LRQ_EINVAL; }
    if (m > 0 && (rc = check_index(d_llrc, d_llrc_blocks, 16))) return rc;
    const OneString<int64_t> src{reinterpret_cast<const longlong2 *>(d_llrc), d_llrc_blocks, n};
    return query_run(src, d_pos, m, mode, d_out, d_offsets, d_recs, capacity, h_total,
                     at<uint32_t>(d_scratch, HDR_ERR), query_sums(d_scratch, m),
                     static_cast<hipStream_t>(stream));
}

}  // extern "C"

// ---- point queries without a caller scratch buffer ------------------------------
//
// lrq_query_multi_noalloc keeps its error word (byte 0) and the all-mode
// scan's tile sums (from byte 256) in this library-owned array, one copy per
// GPU for the life of the process.  In host code the name is only a stand-in
// for the device copy: the address kernels use comes from
// hipGetSymbolAddress, looked up once per device.
constexpr size_t NOALLOC_SUMS_AT = 256;
constexpr size_t NOALLOC_BYTES =
    NOALLOC_SUMS_AT + size_t((LRQ_NOALLOC_MAX_QUERIES + 1 + RS_TILE - 1) / RS_TILE) * 8;
static __device__ __align__(256) uint8_t scratch[(NOALLOC_BYTES + 255) / 256 * 256];

namespace lrq {
namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex noalloc_mu;
void *noalloc_ptr[NOALLOC_MAX_DEVICES];

// The device address of `scratch` on the current device.
int noalloc_scratch(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) { set_error("hipGetDevice: %s", hipGetErrorString(e)); return LRQ_EDEVICE; }
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) { set_error("device %d out of range", dev); return LRQ_EDEVICE; }
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (!noalloc_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            return LRQ_EDEVICE;
        }
        noalloc_ptr[dev] = p;
    }
    *out = noalloc_ptr[dev];
    return LRQ_OK;
}

}  // namespace
}  // namespace lrq

extern "C" {

int lrq_query_multi_noalloc(const lrq_string_ref *d_refs, int32_t nrefs, const int32_t *d_sid,
                            const int32_t *d_pos, int64_t m, int32_t mode, lrq_rec *d_out,
                            int64_t *d_offsets, lrq_rec *d_recs, int64_t capacity,
                            int64_t *h_total, uint32_t *h_errors, void *stream) {
    clear_error();
    if (m > LRQ_NOALLOC_MAX_QUERIES) {
        set_error("m = %lld queries, more than LRQ_NOALLOC_MAX_QUERIES (%lld)", (long long)m,
                  (long long)LRQ_NOALLOC_MAX_QUERIES);
        return LRQ_ERANGE;
    }
    // the same argument checks as lrq_query_multi, against a dummy scratch
    // that passes the scratch checks (the array below replaces it)
    alignas(256) static const uint8_t dummy[256] = {};
    int rc = check_query(0, d_pos, m, mode, d_out, d_offsets, d_recs, capacity,
                         const_cast<uint8_t *>(dummy), size_t(1) << 62);
    if (rc) return rc;
    if (nrefs < 0) { set_error("nrefs < 0"); return LRQ_EINVAL; }
    if (m > 0 && (!d_refs || !d_sid)) { set_error("d_refs / d_sid is NULL"); return LRQ_EINVAL; }
    if (m > 0 && misaligned(d_refs, 8)) { set_error("d_refs not 8-byte aligned"); return LRQ_EINVAL; }
    void *ptr = nullptr;
    if ((rc = noalloc_scratch(&ptr))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint32_t *err = at<uint32_t>(ptr, HDR_ERR);
    // each call's error bits are its own: the word is cleared by a kernel
    // (not a memset, so that the call can be captured in a graph)
    if ((rc = run_zero(reinterpret_cast<uint64_t *>(err), 1, st))) return rc;
    const ManyStrings src{d_refs, nrefs, d_sid};
    rc = query_run(src, d_pos, m, mode, d_out, d_offsets, d_recs, capacity, h_total, err,
                   at<int64_t>(ptr, NOALLOC_SUMS_AT), st);
    if (h_errors && (rc == LRQ_OK || rc == LRQ_ENOSPC)) {
        hipError_t e = hipMemcpyAsync(h_errors, err, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) { set_error("reading the error word: %s", hipGetErrorString(e)); return LRQ_EDEVICE; }
    }
    return rc;
}

}  // extern "C"
