/*
 * lrq.h -- longest-repeat queries on AMD MI355X (gfx950): the C ABI.
 *
 * Computes, for every position k of a string S, the longest repeat covering
 * k (Y. Tian and B. Xu, "On Longest Repeat Queries Using GPU", arXiv
 * 1501.06663; Section 2, Definition 1 and the problem statement), or all of
 * them, through the paper's route: suffix array -> Rank -> LCP -> left-bounded
 * longest repeats (Section 3, Lemma 1) -> compaction of the useless ones
 * (Section 4.2) -> one covering-window scan per position (Sections 4.2, 5.2).
 *
 * Conventions shared by every call
 *   - Positions are 0-based (the paper is 1-based).  A record is
 *     (start, length); "LR_k does not exist" is (-1, 0), the paper's sentinel.
 *   - Characters are bytes; suffix order is unsigned byte order with a proper
 *     prefix first (Section 2).  Any byte value is allowed; no sentinel.
 *   - Sizes: 0 <= total <= LRQ_MAX_TOTAL; positions and lengths are int32.
 *   - Batches: nseg independent strings laid end to end.  seg_off (device,
 *     int64[nseg+1], seg_off[0] = 0, non-decreasing, seg_off[nseg] = total)
 *     delimits them; pass seg_off = NULL and nseg = 1 for one string.  No
 *     repeat crosses a segment boundary; SA values, record starts and query
 *     positions are local to their segment; CSR offsets are global.
 *   - Pointers prefixed d_ are device pointers, h_ host pointers.  Every
 *     buffer is owned by the caller; the library allocates nothing except a
 *     thread-local error string (and holds one fixed device array per GPU
 *     for lrq_query_multi_noalloc).
 *   - stream is a hipStream_t (NULL = the null stream).  Device work is
 *     enqueued asynchronously; only calls that return a host value
 *     (h_total, lrq_read_errors) synchronise the stream.
 *   - Return value: LRQ_OK or a negative lrq_status.  Arguments are checked on
 *     the host before anything is launched; a failed check launches nothing.
 *     Device-side checks (SA values outside their segment, neighbour indices
 *     outside their segment, an all-mode capacity that is too small) never
 *     write out of bounds: they set bits of the error word in the scratch
 *     buffer, read back with lrq_read_errors.  An SA whose values lie in range
 *     but repeat (not a permutation) is not detected: its answers are
 *     unspecified, and every access still stays inside the caller's buffers.
 *   - The scratch buffer (lrq_scratch_bytes) holds counters, look-back
 *     descriptors and seeds.  Calls that share one scratch buffer must be
 *     ordered on one stream.
 *   - The compact index of a string or batch is what the LR calls read:
 *       d_llrc         lrq_rec[total]: the compact LLR array (Section 4.2),
 *                      (start, length) with GLOBAL starts, both strictly
 *                      increasing;
 *       d_llrc_blocks  int64[ceil(total / LRQ_BLOCK) + 1]: entry j is the
 *                      number of compact entries that start before position
 *                      j * LRQ_BLOCK; the last entry is their total.
 *     It is produced by lrq_llr_filter (or lrq_index_build) and stays valid
 *     as long as the caller keeps the two buffers.
 */
#ifndef LRQ_H
#define LRQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LRQ_API_VERSION 4
#define LRQ_MAX_TOTAL 2147483646LL /* int32 positions, and one past the end */
#define LRQ_BLOCK 1024             /* positions per entry of the block table */

typedef struct {
    int32_t start;  /* first position of the repeat (segment-local), or -1 */
    int32_t length; /* its length, or 0 */
} lrq_rec;

/* The same record with 64-bit fields, for the lrq64_ calls (strings and
 * batches beyond LRQ_MAX_TOTAL positions). */
typedef struct {
    int64_t start;
    int64_t length;
} lrq_rec64;
#define LRQ64_MAX_TOTAL (1LL << 40) /* positions of the lrq64_ calls */

/* One resident string inside a compact index (see below): the index buffers,
 * the number of positions the index covers, and where the string lies in it. */
typedef struct {
    const lrq_rec *llrc;    /* device: compact array of the index */
    const int64_t *blocks;  /* device: block table of the index */
    int64_t total;          /* positions covered by the index */
    int64_t begin;          /* the string's first position in the index */
    int64_t length;         /* the string's length */
} lrq_string_ref;

typedef enum {
    LRQ_OK = 0,
    LRQ_EINVAL = -1,   /* null pointer, bad count or flag */
    LRQ_ERANGE = -2,   /* size beyond LRQ_MAX_TOTAL */
    LRQ_ENOSPC = -3,   /* a buffer is smaller than the result */
    LRQ_ENOMEM = -4,   /* scratch buffer smaller than lrq_scratch_bytes */
    LRQ_EDEVICE = -5,  /* a HIP call failed; lrq_last_error() has the detail */
    LRQ_EDATA = -6     /* a device-side input check failed (see LRQ_ERR_*) */
} lrq_status;

enum { LRQ_LEFTMOST = 0, LRQ_ALL = 1 };

/* Bits of the device error word (lrq_read_errors). */
#define LRQ_ERR_SA 1u        /* an SA value outside its segment */
#define LRQ_ERR_PHI 2u       /* a neighbour index outside its segment */
#define LRQ_ERR_TIMEOUT 4u   /* a look-back wait hit its bound */
#define LRQ_ERR_CAPACITY 8u  /* all-mode records beyond the given capacity */
#define LRQ_ERR_QUERY 16u    /* a query position outside its string */
#define LRQ_ERR_WALK 32u     /* a raw-LLR walk exceeded its bound (lrq_lr_*_raw) */

/* ---------------------------------------------------------------- misc -- */

int lrq_version(void);
const char *lrq_status_str(int status);
/* Detail of the last failing call on this thread ("" if none). */
const char *lrq_last_error(void);

/* Device bytes the scratch buffer needs for strings of `total` characters in
 * `nseg` segments (covers every call below). */
int lrq_scratch_bytes(int64_t total, int32_t nseg, size_t *bytes);

/* Kernel shapes.  plcp_chunk: positions one lane walks in the LCP kernel
 * (8, 16 or 32); llr_waves: waves per LLR-filter block (4 or 8); lr_tile:
 * positions per covering-window block (1024, 2048 or 4096); fuse_filter: 1
 * makes lrq_index_build run the LCP walk and the LLR filter as one kernel, 0
 * as two.  Results do not depend on the choice, only speed does.  The setting
 * belongs to the calling thread: every thread starts with the defaults
 * (8, 8, 2048, 0), its calls use its own setting, and threads may change
 * theirs concurrently.  lrq_set_tuning(NULL) restores the defaults.
 * lrq_scratch_bytes covers every allowed tuning. */
typedef struct {
    int32_t plcp_chunk;
    int32_t llr_waves;
    int32_t lr_tile;
    int32_t fuse_filter;
} lrq_tuning;

int lrq_set_tuning(const lrq_tuning *t);
int lrq_get_tuning(lrq_tuning *t);

/* Synchronise `stream`, then return (and clear) the device error word. */
int lrq_read_errors(void *d_scratch, uint32_t *h_flags, void *stream);

/* Per-launch timing.  lrq_timing_start(k) makes the next k kernel launches of
 * the calling thread record a pair of HIP events on their own stream; 0
 * disables.  lrq_timing_collect waits for the recorded events and writes, per
 * launch in order, the kernel name (static string) and its duration in
 * milliseconds; *count gets the number recorded.  The recorder is per thread:
 * launches from other threads are neither recorded nor disturbed. */
int lrq_timing_start(int32_t max_records);
int lrq_timing_collect(int32_t cap, const char **names, float *ms, int32_t *count);
/* Restrict the calling thread's recording to launches of one kernel (its name
 * without template arguments, e.g. "rank_scatter_kernel"), so that the events
 * bracket only that kernel; NULL or "" records every launch again.  The
 * string is copied. */
int lrq_timing_only(const char *kernel);

/* ------------------------------------------- support: suffix array (host) */

/* Suffix array of h_text[0..n) on the host, by induced sorting (SA-IS).  The
 * paper builds SA, Rank and LCP on the host CPU before its GPU kernels and
 * excludes them from its timings (Section 5 opening, Section 6
 * "Measurements"); Section 3 defines SA.  h_sa: caller-owned int32[n]. */
int lrq_build_sa_host(const uint8_t *h_text, int64_t n, int32_t *h_sa);

/* Segment-local suffix arrays of every segment of a batch; h_seg_off is the
 * host copy of the segment offsets.  h_sa: int32[total]. */
int lrq_build_sa_host_batch(const uint8_t *h_text, const int64_t *h_seg_off,
                            int32_t nseg, int32_t *h_sa);

/* ------------------------------------------ support: suffix array (device) */

/* Device bytes of the work buffer lrq_build_sa needs (about 56.3 per character:
 * two 8-byte key arrays, two 4-byte value arrays, eight 4-byte per-suffix
 * arrays, and the per-tile histograms). */
int lrq_sa_work_bytes(int64_t total, int32_t nseg, size_t *bytes);

/* Segment-local suffix arrays on the device, the same result as
 * lrq_build_sa_host[_batch] (Section 3's SA: suffixes in lexicographic order of
 * unsigned bytes, a proper prefix first), by prefix doubling (Manber and
 * Myers, SIAM J. Comput. 1993) over a radix sort.  The paper builds SA on the
 * host and excludes it from its timings; this call moves that step onto the
 * GPU.  d_text: uint8[total], 8-byte aligned; d_seg_off as everywhere (NULL
 * when nseg == 1); d_sa: int32[total]; d_work: lrq_sa_work_bytes bytes,
 * 256-byte aligned, contents not preserved.  The call synchronises `stream`
 * once per doubling round (it reads the number of distinct ranks) and returns
 * when the SA is complete. */
int lrq_build_sa(const uint8_t *d_text, int64_t total, const int64_t *d_seg_off, int32_t nseg,
                 int32_t *d_sa, void *d_work, size_t work_bytes, void *stream);

/* ---------------------------------------------------- the hot path (GPU) */

/*
 * Rank scatter (Section 3: Rank is the inverse of SA; Theorem 1 proof).
 * For every suffix-array slot r of segment b with base o = seg_off[b]:
 *   d_nbr[2*(o+SA[r])]   = o + SA[r-1]  (-1 if r = 0)     -- Phi, the suffix
 *                                          ranked just before
 *   d_nbr[2*(o+SA[r])+1] = o + SA[r+1]  (-1 if r is last)  -- the one after
 *   d_rank[o+SA[r]]      = r            (only if d_rank != NULL)
 * d_sa: int32[total], segment-local values.  d_nbr: int32[2*total], by text
 * position (global).  Lemma 1 needs LCP[Rank[i]] and LCP[Rank[i]+1], the lcp
 * of suffix i with these two neighbours.  SA values outside their segment set
 * LRQ_ERR_SA and are skipped.  Repeated in-range values are not detected; the
 * slots they leave unwritten keep whatever d_nbr held.
 */
int lrq_rank_scatter(const int32_t *d_sa, int64_t total, const int64_t *d_seg_off,
                     int32_t nseg, int32_t *d_nbr, int32_t *d_rank,
                     void *d_scratch, size_t scratch_bytes, void *stream);

/*
 * Text-order LCP (Section 3, the lcp array; Kasai et al. as cited in
 * Theorem 1).  In place over d_pn (int32[2*total]): in, the neighbours of
 * lrq_rank_scatter; out, d_pn[2i] = LCP[Rank[i]] (lcp with the preceding
 * suffix) and d_pn[2i+1] = LCP[Rank[i]+1] (lcp with the following suffix),
 * 0 where the neighbour does not exist (the paper's LCP[1] = LCP[n+1] = 0).
 * d_text: uint8[total].
 */
int lrq_plcp(const uint8_t *d_text, int64_t total, const int64_t *d_seg_off,
             int32_t nseg, int32_t *d_pn, void *d_scratch, size_t scratch_bytes,
             void *stream);

/*
 * LLR filter (Section 3, Lemma 1; compaction of Section 4.2 and the
 * K1-K3 kernels of Section 5.2, fused into one pass).
 *   L_i = max(d_pn[2i], d_pn[2i+1]);  keep i iff L_i > 0 and L_i >= L_{i-1}
 *   (L_{-1} = 0 at every segment start); kept i are written in increasing i
 *   as d_llrc[j] = (i, L_i) with GLOBAL positions i.
 * Outputs the compact index (d_llrc, d_llrc_blocks); *d_llrc_count (device
 * int64) also receives the number of entries.  d_L (int32[total], optional)
 * receives every L_i: the raw LLR array of Section 4.1.  d_pn 16-byte aligned.
 */
int lrq_llr_filter(const int32_t *d_pn, int64_t total, const int64_t *d_seg_off,
                   int32_t nseg, lrq_rec *d_llrc, int64_t *d_llrc_count,
                   int64_t *d_llrc_blocks, int32_t *d_L, void *d_scratch,
                   size_t scratch_bytes, void *stream);

/*
 * The same filter from the paper's own GPU input (Section 5: the Rank and LCP
 * arrays are copied to the device): d_rank int32[n], d_lcp int32[n+1] with
 * d_lcp[0] = d_lcp[n] = 0.  One string.  (LCP[Rank[i]], LCP[Rank[i]+1]) is
 * gathered into d_work (int32[2n], 16-byte aligned), then filtered as above.
 * Rank values outside [0, n) set LRQ_ERR_SA and read as length 0.
 */
int lrq_llr_from_rank_lcp(const int32_t *d_rank, const int32_t *d_lcp, int64_t n,
                          int32_t *d_work, lrq_rec *d_llrc, int64_t *d_llrc_count,
                          int64_t *d_llrc_blocks, int32_t *d_L, void *d_scratch,
                          size_t scratch_bytes, void *stream);

/*
 * Rank scatter + text-order LCP + LLR filter in one call.  d_work:
 * int32[2*total], 16-byte aligned, transient: its contents afterwards are
 * unspecified.  The build may also use d_llrc's buffer (lrq_rec[total]) for
 * the neighbour pairs before it writes the compact array there.  With the
 * filter not fused, the LCP walk hands Lemma 1's L to the filter instead of
 * the (PLCP, NLCP) pairs, through d_L when given (which then holds L, as
 * lrq_llr_filter would leave it), else through d_work.
 */
int lrq_index_build(const uint8_t *d_text, const int32_t *d_sa, int64_t total,
                    const int64_t *d_seg_off, int32_t nseg, int32_t *d_work,
                    lrq_rec *d_llrc, int64_t *d_llrc_count, int64_t *d_llrc_blocks,
                    int32_t *d_L, void *d_scratch, size_t scratch_bytes, void *stream);

/*
 * Leftmost longest repeat of every position (Algorithm 2's result, reading its
 * stop test as "stop at the first entry that starts right of k").  For each
 * global position k the covering entries of the compact array form one
 * contiguous window (starts and ends both increase, Section 4.2); the answer is
 * the longest entry of that window, the smallest start on ties.
 * d_out: lrq_rec[total], 16-byte aligned, starts segment-local.
 */
int lrq_lr_leftmost(const lrq_rec *d_llrc, const int64_t *d_llrc_blocks, int64_t total,
                    const int64_t *d_seg_off, int32_t nseg, lrq_rec *d_out,
                    void *d_scratch, size_t scratch_bytes, void *stream);

/*
 * All longest repeats of every position (Algorithm 4; the problem statement of
 * Section 2 asks for all of them), as CSR: d_offsets int64[total+1] (global,
 * 16-byte aligned) and d_recs (ascending start within each position, starts
 * segment-local).
 *   lrq_lr_all        one pass: counts, offsets and records.  Records at index
 *                     >= capacity are not written and set LRQ_ERR_CAPACITY.
 *                     If h_total != NULL it synchronises, stores the record
 *                     total there and returns LRQ_ENOSPC when it exceeds
 *                     capacity (call again with a larger buffer).
 *   lrq_lr_all_count  the record total only, for sizing the buffer (synchronises
 *                     when h_total != NULL).
 */
int lrq_lr_all(const lrq_rec *d_llrc, const int64_t *d_llrc_blocks, int64_t total,
               const int64_t *d_seg_off, int32_t nseg, int64_t *d_offsets,
               lrq_rec *d_recs, int64_t capacity, int64_t *h_total, void *d_scratch,
               size_t scratch_bytes, void *stream);
int lrq_lr_all_count(const lrq_rec *d_llrc, const int64_t *d_llrc_blocks, int64_t total,
                     const int64_t *d_seg_off, int32_t nseg, int64_t *h_total,
                     void *d_scratch, size_t scratch_bytes, void *stream);

/*
 * The raw-LLR path (Section 4.1, Figure 2's first option; Algorithms 1 and 3):
 * the same answers as lrq_lr_leftmost / lrq_lr_all, computed from the raw LLR
 * array L without the compaction of Section 4.2.
 *   lrq_llr_lengths     Lemma 1 only: d_L[i] = max(d_pn[2i], d_pn[2i+1]) from
 *                       lrq_plcp's pairs.  d_pn 16-byte, d_L 8-byte aligned.
 *   lrq_lr_leftmost_raw for every global position k, the longest LLR that
 *                       covers k, the smallest start on ties; (-1, 0) if none.
 *   lrq_lr_all_raw      every covering LLR of maximal length, ascending start,
 *                       as CSR (offsets, capacity and h_total as lrq_lr_all;
 *                       d_offsets only needs 8-byte alignment here); with
 *                       d_out (optional, lrq_rec[total]) the leftmost records
 *                       too, from the same walks (both modes, as lrq_lr_both).
 * Within a string i + L_i never decreases, so the LLRs covering k are the
 * positions [lo(k), k]; each position walks left over them: O(alpha) work per
 * position, alpha the mean LLR length (Lemma 4), against O(beta) for the
 * compact scans.  The path fits texts whose repeats are short.  A walk longer
 * than max_walk LLRs (<= 0: 65536) stops and sets LRQ_ERR_WALK, and that
 * position's answer is incomplete: use the compact path for such texts.  An
 * LLR that runs past its string sets LRQ_ERR_SA.  d_L: int32[total], the
 * values of lrq_llr_filter's d_L or lrq_llr_lengths; starts in the output
 * are segment-local.
 */
int lrq_llr_lengths(const int32_t *d_pn, int64_t total, int32_t *d_L, void *stream);
int lrq_lr_leftmost_raw(const int32_t *d_L, int64_t total, const int64_t *d_seg_off,
                        int32_t nseg, int32_t max_walk, lrq_rec *d_out, void *d_scratch,
                        size_t scratch_bytes, void *stream);
int lrq_lr_all_raw(const int32_t *d_L, int64_t total, const int64_t *d_seg_off, int32_t nseg,
                   int32_t max_walk, lrq_rec *d_out, int64_t *d_offsets, lrq_rec *d_recs,
                   int64_t capacity, int64_t *h_total, void *d_scratch, size_t scratch_bytes,
                   void *stream);

/*
 * Both answers of Section 2's problem in one pass over the compact array: the
 * leftmost longest repeat of every position into d_out (as lrq_lr_leftmost)
 * and all longest repeats into d_offsets / d_recs (as lrq_lr_all, with the
 * same capacity and h_total contract).  The outputs are identical to those of
 * the two separate calls; the leftmost records are written while each tile
 * waits for its record offset, so the pair costs little more than all mode.
 * d_out: lrq_rec[total], 8-byte aligned (NULL allowed when total == 0).
 */
int lrq_lr_both(const lrq_rec *d_llrc, const int64_t *d_llrc_blocks, int64_t total,
                const int64_t *d_seg_off, int32_t nseg, lrq_rec *d_out, int64_t *d_offsets,
                lrq_rec *d_recs, int64_t capacity, int64_t *h_total, void *d_scratch,
                size_t scratch_bytes, void *stream);

/*
 * Point queries on one string: the answer of Section 2's problem at m given
 * positions only (Algorithm 2 per queried position for the leftmost LR,
 * Algorithm 4 for all of them: find the first covering entry of the compact
 * array, then walk right while entries start at or before k; Section 4.2).
 * The block table narrows the search to the entries near k.  The results are
 * those of lrq_lr_leftmost / lrq_lr_all at the same positions.
 *   d_pos   int32[m], positions in [0, n).  An out-of-range position answers
 *           (-1, 0) / an empty list and sets LRQ_ERR_QUERY.
 *   mode    LRQ_LEFTMOST: d_out lrq_rec[m] (8-byte aligned) gets the leftmost
 *           LR of every query; d_offsets, d_recs, capacity and h_total are
 *           ignored.
 *           LRQ_ALL: CSR over the queries, in query order.  d_offsets
 *           int64[m+1] (8-byte aligned), d_recs lrq_rec[capacity] with the
 *           records of query q at [d_offsets[q], d_offsets[q+1]) in ascending
 *           start; records at index >= capacity are not written and set
 *           LRQ_ERR_CAPACITY.  d_out (optional, lrq_rec[m]) also receives the
 *           leftmost records.  If h_total != NULL the call synchronises,
 *           stores the record total there and returns LRQ_ENOSPC when it
 *           exceeds capacity (call again with a larger buffer).
 *   scratch leftmost: lrq_scratch_bytes(n, 1) bytes; all mode:
 *           lrq_scratch_bytes(max(n, m), 1) bytes (it holds the scan of the
 *           m counts).
 * Starts are local to the string (the index's own positions here).
 */
int lrq_query_positions(const lrq_rec *d_llrc, const int64_t *d_llrc_blocks, int64_t n,
                        const int32_t *d_pos, int64_t m, int32_t mode, lrq_rec *d_out,
                        int64_t *d_offsets, lrq_rec *d_recs, int64_t capacity, int64_t *h_total,
                        void *d_scratch, size_t scratch_bytes, void *stream);

/*
 * Point queries on many resident strings in one launch chain (the same
 * per-position search and the same modes, outputs and capacity contract as
 * lrq_query_positions).  Query q asks for position d_pos[q] of string
 * d_sid[q]; d_refs (device, lrq_string_ref[nrefs], 8-byte aligned) describes
 * the strings, which may live in different indexes.  A string id outside
 * [0, nrefs) or a position outside [0, length) answers (-1, 0) / an empty list
 * and sets LRQ_ERR_QUERY.  Starts are local to the string.  Scratch:
 * lrq_scratch_bytes(0, 1) bytes for leftmost mode, lrq_scratch_bytes(m, 1)
 * for all mode.  The referenced index buffers must stay valid until the
 * launches complete.
 */
int lrq_query_multi(const lrq_string_ref *d_refs, int32_t nrefs, const int32_t *d_sid,
                    const int32_t *d_pos, int64_t m, int32_t mode, lrq_rec *d_out,
                    int64_t *d_offsets, lrq_rec *d_recs, int64_t capacity, int64_t *h_total,
                    void *d_scratch, size_t scratch_bytes, void *stream);

/* ------------------------------------ 64-bit positions (lrq64_ calls) -- */

/*
 * The hot path with 64-bit positions and lengths, for strings and batches of
 * more than LRQ_MAX_TOTAL characters (up to LRQ64_MAX_TOTAL; the paper's
 * scalability discussion, Section 6, runs the same queries on larger inputs).
 * Each call computes exactly what its 32-bit namesake computes (same
 * sections of the paper), with every position, SA value, neighbour, lcp and
 * length an int64 and every record an lrq_rec64; counts, offsets, the block
 * table, the error word and the calling conventions are unchanged.  Buffers
 * of pairs (d_nbr, d_pn, d_work, compact array, records) are 16-byte aligned,
 * d_L too.  The build (lrq64_index_build) always runs the LCP walk and the
 * filter as two kernels, the filter with its own look-back (the fused-filter
 * tuning does not apply).  The scratch buffer: lrq64_scratch_bytes bytes,
 * which equals lrq_scratch_bytes where both are defined.  Not provided with
 * 64-bit positions: the raw-LLR path, the paper-input filter, the device and
 * host suffix-array builders and the multi-string point query.
 */
int lrq64_scratch_bytes(int64_t total, int32_t nseg, size_t *bytes);
int lrq64_rank_scatter(const int64_t *d_sa, int64_t total, const int64_t *d_seg_off,
                       int32_t nseg, int64_t *d_nbr, int64_t *d_rank, void *d_scratch,
                       size_t scratch_bytes, void *stream);
int lrq64_plcp(const uint8_t *d_text, int64_t total, const int64_t *d_seg_off, int32_t nseg,
               int64_t *d_pn, void *d_scratch, size_t scratch_bytes, void *stream);
int lrq64_llr_filter(const int64_t *d_pn, int64_t total, const int64_t *d_seg_off, int32_t nseg,
                     lrq_rec64 *d_llrc, int64_t *d_llrc_count, int64_t *d_llrc_blocks,
                     int64_t *d_L, void *d_scratch, size_t scratch_bytes, void *stream);
int lrq64_index_build(const uint8_t *d_text, const int64_t *d_sa, int64_t total,
                      const int64_t *d_seg_off, int32_t nseg, int64_t *d_work, lrq_rec64 *d_llrc,
                      int64_t *d_llrc_count, int64_t *d_llrc_blocks, int64_t *d_L,
                      void *d_scratch, size_t scratch_bytes, void *stream);
int lrq64_lr_leftmost(const lrq_rec64 *d_llrc, const int64_t *d_llrc_blocks, int64_t total,
                      const int64_t *d_seg_off, int32_t nseg, lrq_rec64 *d_out, void *d_scratch,
                      size_t scratch_bytes, void *stream);
int lrq64_lr_all_count(const lrq_rec64 *d_llrc, const int64_t *d_llrc_blocks, int64_t total,
                       const int64_t *d_seg_off, int32_t nseg, int64_t *h_total, void *d_scratch,
                       size_t scratch_bytes, void *stream);
int lrq64_lr_all(const lrq_rec64 *d_llrc, const int64_t *d_llrc_blocks, int64_t total,
                 const int64_t *d_seg_off, int32_t nseg, int64_t *d_offsets, lrq_rec64 *d_recs,
                 int64_t capacity, int64_t *h_total, void *d_scratch, size_t scratch_bytes,
                 void *stream);
int lrq64_lr_both(const lrq_rec64 *d_llrc, const int64_t *d_llrc_blocks, int64_t total,
                  const int64_t *d_seg_off, int32_t nseg, lrq_rec64 *d_out, int64_t *d_offsets,
                  lrq_rec64 *d_recs, int64_t capacity, int64_t *h_total, void *d_scratch,
                  size_t scratch_bytes, void *stream);
/* Point queries on one string; d_pos int64[m]. */
int lrq64_query_positions(const lrq_rec64 *d_llrc, const int64_t *d_llrc_blocks, int64_t n,
                          const int64_t *d_pos, int64_t m, int32_t mode, lrq_rec64 *d_out,
                          int64_t *d_offsets, lrq_rec64 *d_recs, int64_t capacity,
                          int64_t *h_total, void *d_scratch, size_t scratch_bytes, void *stream);

/*
 * lrq_query_multi for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * The same queries, modes, outputs and capacity contract as lrq_query_multi,
 * without the scratch argument: the error word and the all-mode scan's partial
 * sums live in a library-owned device array of about 33 KB, one per GPU,
 * held from the first call on that GPU until the process ends.  The call
 * allocates nothing (no hipMalloc, no allocating library routine).
 *   m          at most LRQ_NOALLOC_MAX_QUERIES; more gives LRQ_ERANGE before
 *              anything is launched.
 *   h_errors   optional host uint32: when given, the call synchronises
 *              `stream` and stores the device error bits of this call
 *              (LRQ_ERR_QUERY, LRQ_ERR_CAPACITY); each call clears the
 *              array's error word when it starts.
 * Every call on one GPU uses that GPU's one array and leaves its contents
 * behind: calls that overlap in time on one GPU (other streams, other threads)
 * race on it and must be ordered by the caller.  The current device must be
 * the device of `stream` and of every buffer.
 */
#define LRQ_NOALLOC_MAX_QUERIES (1LL << 24)
int lrq_query_multi_noalloc(const lrq_string_ref *d_refs, int32_t nrefs, const int32_t *d_sid,
                            const int32_t *d_pos, int64_t m, int32_t mode, lrq_rec *d_out,
                            int64_t *d_offsets, lrq_rec *d_recs, int64_t capacity,
                            int64_t *h_total, uint32_t *h_errors, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* LRQ_H */
