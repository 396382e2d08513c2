// Shared host-side definitions of liblrq: scratch-buffer layout, tile sizes,
// the per-thread error string.  Included by the HIP translation unit and the
// host-only one.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>

#include "lrq.h"

namespace lrq {

// ---- tile geometry ---------------------------------------------------------

// Tunable shapes (chosen per workload by the autotuner; defaults below).
//   plcp_chunk  positions one lane walks in the LCP kernel (8, 16, 32); a block
//               always spans 4096 positions, so it has 4096 / plcp_chunk lanes.
//   llr_waves   waves per LLR-filter block (4 or 8); a wave spans 1024
//               positions (one block-table entry).
//   lr_tile     positions per covering-window block (1024, 2048, 4096); 256
//               lanes, lr_tile / 256 positions each.
//   fuse_filter 1: lrq_index_build runs the LCP walk and the LLR filter as one
//               kernel (saves a round trip through the pair array, but its tile
//               look-back makes blocks wait for slower neighbours); 0: two kernels.
struct Tuning {
    int32_t plcp_chunk = 8;
    int32_t llr_waves = 8;
    int32_t lr_tile = 2048;
    int32_t fuse_filter = 0;
};
Tuning &tuning();  // the calling thread's setting (lrq_set_tuning)
bool tuning_valid(const Tuning &t);

// LCP heads: level l holds every (plcp_chunk * PLCP_FANOUT^l)-th position; the
// coarsest level keeps at most PLCP_TOP_HEADS heads.  Its heads are computed
// without a seed, one workgroup each, so the limit trades parallelism (more
// workgroups) against unseeded compares: 4096 keeps the chip busy on the
// largest inputs (a 1024 limit left 171 workgroups on a 90M-character batch).
constexpr int PLCP_SPAN = 4096;
constexpr int PLCP_FANOUT = 16;
constexpr int PLCP_TOP_HEADS = 4096;
constexpr int PLCP_MAX_LEVELS = 8;

// LLR filter: each lane loads 8 x 16 bytes (2 positions per load), so a wave
// spans 8 * 64 * 2 = 1024 positions = one LRQ_BLOCK of the block table.
constexpr int LLR_LOADS = 8;
constexpr int LLR_WAVE_SPAN = LLR_LOADS * 64 * 2;
static_assert(LLR_WAVE_SPAN == LRQ_BLOCK, "one wave span per block-table entry");

// Covering-window scan: 256 lanes per block.
constexpr int LR_THREADS = 256;

// ---- scratch layout --------------------------------------------------------

// Header words (byte offsets).
constexpr size_t HDR_ERR = 0;         // uint32 error bits
constexpr size_t HDR_ALL_TOTAL = 8;   // int64 all-mode record total
constexpr size_t HDR_ALPHA = 16;      // uint32[8]: byte values present in the text
constexpr size_t HDR_SYM_LG = 48;     // int32: log2 of the bits per packed symbol (3 = bytes)
constexpr size_t HDR_BYTES = 256;

// Packed text for the LCP kernels: symbols of 1, 2 or 4 bits when the text
// has at most 2, 4 or 16 distinct byte values (an equality-preserving code),
// stored LSB-first in 64-bit words.  Room for 4-bit symbols plus two words of
// padding, so that a two-word window never leaves the buffer.
inline int64_t packed_words(int64_t total) { return (total + 15) / 16 + 2; }

struct Layout {
    int64_t llr_tiles = 0;
    size_t llr_state = 0;         // uint64[1 + llr_tiles]: tile ticket, then
                                  // one look-back descriptor per tile
    int64_t lr_tiles = 0;
    size_t lr_state = 0;          // uint64[1 + lr_tiles]: ticket + descriptors
    int64_t plcp_tiles = 0;
    size_t plcp_state = 0;        // uint64[2 + 3 * plcp_tiles]: the fused LCP +
                                  // filter's ticket and descriptors, or the
                                  // per-block keep summaries (int4, from word 2)
                                  // and compact-array bases of the unfused path
    int levels = 0;               // head levels 1..levels
    int64_t stride[PLCP_MAX_LEVELS + 1] = {};
    int64_t nheads[PLCP_MAX_LEVELS + 1] = {};
    size_t heads[PLCP_MAX_LEVELS + 1] = {};  // (PLCP, NLCP) pairs, 16 bytes each (room for
                                             // the 64-bit calls)
    size_t packed = 0;            // uint64[packed_words(total)]: packed text
    size_t bytes = 0;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline Layout layout(int64_t total, int32_t nseg, const Tuning &tu) {
    (void)nseg;
    Layout L;
    size_t at = HDR_BYTES;
    const int64_t llr_tile = int64_t(tu.llr_waves) * LLR_WAVE_SPAN;
    L.llr_tiles = (total + llr_tile - 1) / llr_tile;
    L.llr_state = at;
    at = align256(at + size_t(1 + L.llr_tiles) * 8);
    L.lr_tiles = (total + tu.lr_tile - 1) / tu.lr_tile;
    L.lr_state = at;
    at = align256(at + size_t(1 + L.lr_tiles) * 8);
    L.plcp_tiles = (total + PLCP_SPAN - 1) / PLCP_SPAN;
    L.plcp_state = at;
    at = align256(at + size_t(2 + 3 * L.plcp_tiles) * 8);
    int64_t s = tu.plcp_chunk;
    int lv = 0;
    while (lv < PLCP_MAX_LEVELS) {
        s *= PLCP_FANOUT;
        ++lv;
        L.stride[lv] = s;
        L.nheads[lv] = total > 0 ? (total + s - 1) / s : 0;
        L.heads[lv] = at;
        at = align256(at + size_t(L.nheads[lv] > 0 ? L.nheads[lv] : 1) * 16);
        if (L.nheads[lv] <= PLCP_TOP_HEADS) break;
    }
    L.levels = lv;
    L.packed = at;
    at = align256(at + size_t(packed_words(total)) * 8);
    L.bytes = at;
    return L;
}

inline Layout layout(int64_t total, int32_t nseg) { return layout(total, nseg, tuning()); }

// Scratch bytes that fit every allowed tuning (so the tuning can change
// between calls without reallocating).
inline size_t scratch_bytes_any(int64_t total, int32_t nseg) {
    size_t b = 0;
    for (int c : {8, 16, 32})
        for (int w : {4, 8})
            for (int t : {1024, 2048, 4096}) {
                Tuning tu;
                tu.plcp_chunk = c;
                tu.llr_waves = w;
                tu.lr_tile = t;  // fuse_filter does not change the layout
                const size_t x = layout(total, nseg, tu).bytes;
                if (x > b) b = x;
            }
    return b;
}

// ---- errors ----------------------------------------------------------------

void set_error(const char *fmt, ...);
void clear_error();

}  // namespace lrq
