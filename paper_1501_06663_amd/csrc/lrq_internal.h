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

// Text-order LCP: one lane walks a chunk of PLCP_CHUNK consecutive positions
// (Kasai's bound carried inside the chunk); chunk heads are seeded from heads
// of coarser levels, level l holding every (PLCP_CHUNK * PLCP_FANOUT^l)-th
// position.  The coarsest level keeps at most PLCP_TOP_HEADS heads.
constexpr int PLCP_THREADS = 256;
constexpr int PLCP_CHUNK = 16;
constexpr int PLCP_FANOUT = 16;
constexpr int PLCP_TOP_HEADS = 1024;
constexpr int PLCP_MAX_LEVELS = 8;

// LLR filter: 4 waves per block, each wave 8 loads of 16 B (2 positions) per
// lane, so a tile is 4 * 8 * 64 * 2 = 4096 positions and a wave span is one
// LRQ_BLOCK of the block table.
constexpr int LLR_THREADS = 256;
constexpr int LLR_LOADS = 8;
constexpr int LLR_WAVE_SPAN = LLR_LOADS * 64 * 2;
constexpr int LLR_TILE = (LLR_THREADS / 64) * LLR_WAVE_SPAN;
static_assert(LLR_WAVE_SPAN == LRQ_BLOCK, "one wave span per block-table entry");

// Covering-window scan: a tile of LR_TILE positions, LR_PER_THREAD consecutive
// positions per lane; the window of compact entries is staged in LDS when it
// holds at most LR_WINDOW entries.
constexpr int LR_THREADS = 256;
constexpr int LR_PER_THREAD = 8;
constexpr int LR_TILE = LR_THREADS * LR_PER_THREAD;
constexpr int LR_WINDOW = LR_TILE;
static_assert(LR_TILE % LRQ_BLOCK == 0, "LR tiles start on block-table boundaries");

// ---- scratch layout --------------------------------------------------------

// Header words (byte offsets).
constexpr size_t HDR_ERR = 0;         // uint32 error bits
constexpr size_t HDR_ALL_TOTAL = 8;   // int64 all-mode record total
constexpr size_t HDR_BYTES = 256;

struct Layout {
    int64_t llr_tiles = 0;
    size_t llr_state = 0;         // uint64[1 + llr_tiles]: tile ticket, then
                                  // one look-back descriptor per tile
    int64_t lr_tiles = 0;
    size_t lr_state = 0;          // uint64[1 + lr_tiles]: ticket + descriptors
    int levels = 0;               // head levels 1..levels
    int64_t stride[PLCP_MAX_LEVELS + 1] = {};
    int64_t nheads[PLCP_MAX_LEVELS + 1] = {};
    size_t heads[PLCP_MAX_LEVELS + 1] = {};  // int2[nheads]
    size_t bytes = 0;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline Layout layout(int64_t total, int32_t nseg) {
    (void)nseg;
    Layout L;
    size_t at = HDR_BYTES;
    L.llr_tiles = (total + LLR_TILE - 1) / LLR_TILE;
    L.llr_state = at;
    at = align256(at + size_t(1 + L.llr_tiles) * 8);
    L.lr_tiles = (total + LR_TILE - 1) / LR_TILE;
    L.lr_state = at;
    at = align256(at + size_t(1 + L.lr_tiles) * 8);
    int64_t s = PLCP_CHUNK;
    int lv = 0;
    while (lv < PLCP_MAX_LEVELS) {
        s *= PLCP_FANOUT;
        ++lv;
        L.stride[lv] = s;
        L.nheads[lv] = total > 0 ? (total + s - 1) / s : 0;
        L.heads[lv] = at;
        at = align256(at + size_t(L.nheads[lv] > 0 ? L.nheads[lv] : 1) * 8);
        if (L.nheads[lv] <= PLCP_TOP_HEADS) break;
    }
    L.levels = lv;
    L.bytes = at;
    return L;
}

// ---- errors ----------------------------------------------------------------

void set_error(const char *fmt, ...);
void clear_error();

}  // namespace lrq
