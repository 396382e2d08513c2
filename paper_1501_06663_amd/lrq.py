"""Thin Python binding of liblrq (include/lrq.h).

Functions carry the C names without the ``lrq_`` prefix and only marshal
arguments: torch tensors become device pointers, the stream defaults to
torch's current stream, and a non-zero status raises :class:`LrqError`.
Every step of the query runs in the HIP kernels of liblrq; nothing here
computes any part of the answer.  Importing this module fails loudly when
liblrq.so has not been built.

:class:`Index` is a convenience owner of the device buffers for one string
or one batch: it allocates them with torch and calls the C entry points in
order.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblrq.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lrq.h")

LEFTMOST, ALL = 0, 1
ERR_SA, ERR_PHI, ERR_TIMEOUT, ERR_CAPACITY, ERR_QUERY, ERR_WALK = 1, 2, 4, 8, 16, 32
MAX_TOTAL = 2147483646
BLOCK = 1024


def block_entries(total: int) -> int:
    """Length of the block table of a compact index over `total` positions."""
    return (total + BLOCK - 1) // BLOCK + 1


class LrqError(RuntimeError):
    def __init__(self, status: int, call: str, detail: str):
        self.status = status
        super().__init__("%s failed (%d): %s" % (call, status, detail))


def _load():
    # torch brings its own HIP runtime; loading it first makes liblrq's
    # libamdhip64.so.7 dependency bind to that same runtime, so torch's streams
    # and allocations are valid handles inside liblrq (one runtime per process).
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError("liblrq.so is not built (run: python -m paper_1501_06663_amd.build)")
    lib = C.CDLL(LIB_PATH)
    vp, i64, i32, sz = C.c_void_p, C.c_int64, C.c_int32, C.c_size_t
    sigs = {
        "lrq_version": [],
        "lrq_status_str": [C.c_int],
        "lrq_last_error": [],
        "lrq_scratch_bytes": [i64, i32, C.POINTER(sz)],
        "lrq_read_errors": [vp, C.POINTER(C.c_uint32), vp],
        "lrq_build_sa_host": [vp, i64, vp],
        "lrq_build_sa_host_batch": [vp, vp, i32, vp],
        "lrq_sa_work_bytes": [i64, i32, C.POINTER(sz)],
        "lrq_build_sa": [vp, i64, vp, i32, vp, vp, sz, vp],
        "lrq_rank_scatter": [vp, i64, vp, i32, vp, vp, vp, sz, vp],
        "lrq_plcp": [vp, i64, vp, i32, vp, vp, sz, vp],
        "lrq_llr_filter": [vp, i64, vp, i32, vp, vp, vp, vp, vp, sz, vp],
        "lrq_llr_from_rank_lcp": [vp, vp, i64, vp, vp, vp, vp, vp, vp, sz, vp],
        "lrq_index_build": [vp, vp, i64, vp, i32, vp, vp, vp, vp, vp, vp, sz, vp],
        "lrq_lr_leftmost": [vp, vp, i64, vp, i32, vp, vp, sz, vp],
        "lrq_lr_all_count": [vp, vp, i64, vp, i32, C.POINTER(i64), vp, sz, vp],
        "lrq_lr_all": [vp, vp, i64, vp, i32, vp, vp, i64, C.POINTER(i64), vp, sz, vp],
        "lrq_lr_both": [vp, vp, i64, vp, i32, vp, vp, vp, i64, C.POINTER(i64), vp, sz, vp],
        "lrq_llr_lengths": [vp, i64, vp, vp],
        "lrq_lr_leftmost_raw": [vp, i64, vp, i32, i32, vp, vp, sz, vp],
        "lrq_lr_all_raw": [vp, i64, vp, i32, i32, vp, vp, vp, i64, C.POINTER(i64), vp, sz, vp],
        "lrq_query_positions": [vp, vp, i64, vp, i64, i32, vp, vp, vp, i64, C.POINTER(i64), vp,
                                sz, vp],
        "lrq_query_multi": [vp, i32, vp, vp, i64, i32, vp, vp, vp, i64, C.POINTER(i64), vp, sz,
                            vp],
        "lrq_query_multi_noalloc": [vp, i32, vp, vp, i64, i32, vp, vp, vp, i64, C.POINTER(i64),
                                    C.POINTER(C.c_uint32), vp],
        "lrq64_scratch_bytes": [i64, i32, C.POINTER(sz)],
        "lrq64_rank_scatter": [vp, i64, vp, i32, vp, vp, vp, sz, vp],
        "lrq64_plcp": [vp, i64, vp, i32, vp, vp, sz, vp],
        "lrq64_llr_filter": [vp, i64, vp, i32, vp, vp, vp, vp, vp, sz, vp],
        "lrq64_index_build": [vp, vp, i64, vp, i32, vp, vp, vp, vp, vp, vp, sz, vp],
        "lrq64_lr_leftmost": [vp, vp, i64, vp, i32, vp, vp, sz, vp],
        "lrq64_lr_all_count": [vp, vp, i64, vp, i32, C.POINTER(i64), vp, sz, vp],
        "lrq64_lr_all": [vp, vp, i64, vp, i32, vp, vp, i64, C.POINTER(i64), vp, sz, vp],
        "lrq64_lr_both": [vp, vp, i64, vp, i32, vp, vp, vp, i64, C.POINTER(i64), vp, sz, vp],
        "lrq64_query_positions": [vp, vp, i64, vp, i64, i32, vp, vp, vp, i64, C.POINTER(i64), vp,
                                  sz, vp],
        "lrq_set_tuning": [vp],
        "lrq_get_tuning": [vp],
        "lrq_timing_start": [i32],
        "lrq_timing_only": [C.c_char_p],
        "lrq_timing_collect": [i32, C.POINTER(C.c_char_p), C.POINTER(C.c_float), C.POINTER(i32)],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.lrq_status_str.restype = C.c_char_p
    lib.lrq_last_error.restype = C.c_char_p
    return lib


_lib = _load()


def header_functions() -> Sequence[str]:
    """Names of the functions include/lrq.h declares."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(lrq_\w+)\s*\(", text, re.M)))


def _check(rc: int, call: str):
    if rc != 0:
        raise LrqError(rc, call, (_lib.lrq_last_error() or b"").decode())


def _p(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream):
    if stream is not None:
        return stream if isinstance(stream, int) else stream.cuda_stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def _nseg(seg_off, nseg):
    if seg_off is None:
        return 1
    return int(nseg) if nseg is not None else int(seg_off.numel()) - 1


# ---------------------------------------------------------------- C calls --

def version() -> int:
    return int(_lib.lrq_version())


def status_str(status: int) -> str:
    return _lib.lrq_status_str(status).decode()


def scratch_bytes(total: int, nseg: int = 1) -> int:
    out = C.c_size_t()
    _check(_lib.lrq_scratch_bytes(total, nseg, C.byref(out)), "lrq_scratch_bytes")
    return int(out.value)


def read_errors(scratch, stream=None) -> int:
    out = C.c_uint32()
    _check(_lib.lrq_read_errors(_p(scratch), C.byref(out), _stream(stream)), "lrq_read_errors")
    return int(out.value)


def build_sa_host(text: np.ndarray) -> np.ndarray:
    text = np.ascontiguousarray(text, dtype=np.uint8)
    sa = np.empty(len(text), dtype=np.int32)
    _check(_lib.lrq_build_sa_host(_p(text), len(text), _p(sa)), "lrq_build_sa_host")
    return sa


def build_sa_host_batch(text: np.ndarray, seg_off: np.ndarray) -> np.ndarray:
    text = np.ascontiguousarray(text, dtype=np.uint8)
    seg_off = np.ascontiguousarray(seg_off, dtype=np.int64)
    sa = np.empty(len(text), dtype=np.int32)
    _check(_lib.lrq_build_sa_host_batch(_p(text), _p(seg_off), len(seg_off) - 1, _p(sa)),
           "lrq_build_sa_host_batch")
    return sa


def sa_work_bytes(total: int, nseg: int = 1) -> int:
    out = C.c_size_t(0)
    _check(_lib.lrq_sa_work_bytes(total, nseg, C.byref(out)), "lrq_sa_work_bytes")
    return int(out.value)


def build_sa(text, total, seg_off, nseg, sa, work, stream=None):
    """Suffix array on the device (segment-local values), into `sa`."""
    _check(_lib.lrq_build_sa(_p(text), total, _p(seg_off), _nseg(seg_off, nseg), _p(sa), _p(work),
                             work.numel(), _stream(stream)), "lrq_build_sa")


def build_sa_device(text, seg_off=None, stream=None):
    """Allocate and build the suffix array of a device text (uint8 tensor)."""
    import torch
    total = int(text.numel())
    nseg = 1 if seg_off is None else int(seg_off.numel()) - 1
    sa = torch.empty(max(total, 1), dtype=torch.int32, device=text.device)
    work = torch.empty(sa_work_bytes(total, nseg), dtype=torch.uint8, device=text.device)
    build_sa(text, total, seg_off, nseg, sa, work, stream)
    return sa[:total]


def rank_scatter(sa, total, seg_off, nseg, nbr, rank, scratch, stream=None):
    _check(_lib.lrq_rank_scatter(_p(sa), total, _p(seg_off), _nseg(seg_off, nseg), _p(nbr),
                                 _p(rank), _p(scratch), scratch.numel(), _stream(stream)),
           "lrq_rank_scatter")


def plcp(text, total, seg_off, nseg, pn, scratch, stream=None):
    _check(_lib.lrq_plcp(_p(text), total, _p(seg_off), _nseg(seg_off, nseg), _p(pn),
                         _p(scratch), scratch.numel(), _stream(stream)), "lrq_plcp")


def llr_filter(pn, total, seg_off, nseg, llrc, count, blocks, L, scratch, stream=None):
    _check(_lib.lrq_llr_filter(_p(pn), total, _p(seg_off), _nseg(seg_off, nseg), _p(llrc),
                               _p(count), _p(blocks), _p(L), _p(scratch), scratch.numel(),
                               _stream(stream)), "lrq_llr_filter")


def llr_from_rank_lcp(rank, lcp, n, work, llrc, count, blocks, L, scratch, stream=None):
    _check(_lib.lrq_llr_from_rank_lcp(_p(rank), _p(lcp), n, _p(work), _p(llrc), _p(count),
                                      _p(blocks), _p(L), _p(scratch), scratch.numel(),
                                      _stream(stream)), "lrq_llr_from_rank_lcp")


def index_build(text, sa, total, seg_off, nseg, work, llrc, count, blocks, L, scratch,
                stream=None):
    _check(_lib.lrq_index_build(_p(text), _p(sa), total, _p(seg_off), _nseg(seg_off, nseg),
                                _p(work), _p(llrc), _p(count), _p(blocks), _p(L), _p(scratch),
                                scratch.numel(), _stream(stream)), "lrq_index_build")


def lr_leftmost(llrc, blocks, total, seg_off, nseg, out, scratch, stream=None):
    _check(_lib.lrq_lr_leftmost(_p(llrc), _p(blocks), total, _p(seg_off), _nseg(seg_off, nseg),
                                _p(out), _p(scratch), scratch.numel(), _stream(stream)),
           "lrq_lr_leftmost")


def lr_all_count(llrc, blocks, total, seg_off, nseg, scratch, stream=None, want_total=True):
    out = C.c_int64(-1)
    _check(_lib.lrq_lr_all_count(_p(llrc), _p(blocks), total, _p(seg_off), _nseg(seg_off, nseg),
                                 C.byref(out) if want_total else None, _p(scratch),
                                 scratch.numel(), _stream(stream)), "lrq_lr_all_count")
    return int(out.value)


def lr_all(llrc, blocks, total, seg_off, nseg, offsets, recs, capacity, scratch, stream=None,
           want_total=True):
    """One-pass all mode; returns the record total (-1 without want_total)."""
    out = C.c_int64(-1)
    _check(_lib.lrq_lr_all(_p(llrc), _p(blocks), total, _p(seg_off), _nseg(seg_off, nseg),
                           _p(offsets), _p(recs), capacity, C.byref(out) if want_total else None,
                           _p(scratch), scratch.numel(), _stream(stream)), "lrq_lr_all")
    return int(out.value)


def lr_both(llrc, blocks, total, seg_off, nseg, out, offsets, recs, capacity, scratch, stream=None,
            want_total=True):
    """Leftmost and all modes in one pass; returns the record total (-1
    without want_total)."""
    tot = C.c_int64(-1)
    _check(_lib.lrq_lr_both(_p(llrc), _p(blocks), total, _p(seg_off), _nseg(seg_off, nseg), _p(out),
                            _p(offsets), _p(recs), capacity, C.byref(tot) if want_total else None,
                            _p(scratch), scratch.numel(), _stream(stream)), "lrq_lr_both")
    return int(tot.value)


def llr_lengths(pn, total, L, stream=None):
    """Lemma 1: L[i] = max of the pair (PLCP[i], NLCP[i]) in pn."""
    _check(_lib.lrq_llr_lengths(_p(pn), total, _p(L), _stream(stream)), "lrq_llr_lengths")


def lr_leftmost_raw(L, total, seg_off, nseg, out, scratch, stream=None, max_walk=0):
    """Leftmost LR of every position from the raw LLR array (Algorithm 1)."""
    _check(_lib.lrq_lr_leftmost_raw(_p(L), total, _p(seg_off), _nseg(seg_off, nseg), max_walk,
                                    _p(out), _p(scratch), scratch.numel(), _stream(stream)),
           "lrq_lr_leftmost_raw")


def lr_all_raw(L, total, seg_off, nseg, offsets, recs, capacity, scratch, stream=None,
               max_walk=0, want_total=True, out=None):
    """All LRs of every position from the raw LLR array (Algorithm 3), CSR,
    and with `out` the leftmost records too; returns the record total (-1
    without want_total)."""
    tot = C.c_int64(-1)
    _check(_lib.lrq_lr_all_raw(_p(L), total, _p(seg_off), _nseg(seg_off, nseg), max_walk,
                               _p(out), _p(offsets), _p(recs), capacity,
                               C.byref(tot) if want_total else None, _p(scratch), scratch.numel(),
                               _stream(stream)), "lrq_lr_all_raw")
    return int(tot.value)


def query_positions(llrc, blocks, n, pos, m, out, scratch, stream=None, mode=LEFTMOST,
                    offsets=None, recs=None, capacity=0, want_total=True):
    """Point queries on one string.  Leftmost mode fills `out`; all mode fills
    the CSR (offsets, recs) and, with `out`, the leftmost records too, and
    returns the record total (-1 without want_total)."""
    tot = C.c_int64(-1)
    _check(_lib.lrq_query_positions(_p(llrc), _p(blocks), n, _p(pos), m, mode, _p(out),
                                    _p(offsets), _p(recs), capacity,
                                    C.byref(tot) if (want_total and mode == ALL) else None,
                                    _p(scratch), scratch.numel(), _stream(stream)),
           "lrq_query_positions")
    return int(tot.value)


class StringRef(C.Structure):
    """lrq_string_ref: one resident string inside a compact index."""
    _fields_ = [("llrc", C.c_void_p), ("blocks", C.c_void_p), ("total", C.c_int64),
                ("begin", C.c_int64), ("length", C.c_int64)]


REF_WORDS = C.sizeof(StringRef) // 8   # int64 words per lrq_string_ref


def query_multi(refs, nrefs, sid, pos, m, out, scratch, stream=None, mode=LEFTMOST, offsets=None,
                recs=None, capacity=0, want_total=True):
    """refs: device int64 tensor holding nrefs packed lrq_string_ref records.
    Modes and outputs as query_positions."""
    tot = C.c_int64(-1)
    _check(_lib.lrq_query_multi(_p(refs), nrefs, _p(sid), _p(pos), m, mode, _p(out), _p(offsets),
                                _p(recs), capacity,
                                C.byref(tot) if (want_total and mode == ALL) else None,
                                _p(scratch), scratch.numel(), _stream(stream)), "lrq_query_multi")
    return int(tot.value)


# ------------------------------------------------ 64-bit positions (lrq64_) --

MAX_TOTAL64 = 1 << 40


def scratch_bytes64(total: int, nseg: int = 1) -> int:
    out = C.c_size_t()
    _check(_lib.lrq64_scratch_bytes(total, nseg, C.byref(out)), "lrq64_scratch_bytes")
    return int(out.value)


def rank_scatter64(sa, total, seg_off, nseg, nbr, rank, scratch, stream=None):
    _check(_lib.lrq64_rank_scatter(_p(sa), total, _p(seg_off), _nseg(seg_off, nseg), _p(nbr),
                                   _p(rank), _p(scratch), scratch.numel(), _stream(stream)),
           "lrq64_rank_scatter")


def plcp64(text, total, seg_off, nseg, pn, scratch, stream=None):
    _check(_lib.lrq64_plcp(_p(text), total, _p(seg_off), _nseg(seg_off, nseg), _p(pn),
                           _p(scratch), scratch.numel(), _stream(stream)), "lrq64_plcp")


def llr_filter64(pn, total, seg_off, nseg, llrc, count, blocks, L, scratch, stream=None):
    _check(_lib.lrq64_llr_filter(_p(pn), total, _p(seg_off), _nseg(seg_off, nseg), _p(llrc),
                                 _p(count), _p(blocks), _p(L), _p(scratch), scratch.numel(),
                                 _stream(stream)), "lrq64_llr_filter")


def index_build64(text, sa, total, seg_off, nseg, work, llrc, count, blocks, L, scratch,
                  stream=None):
    _check(_lib.lrq64_index_build(_p(text), _p(sa), total, _p(seg_off), _nseg(seg_off, nseg),
                                  _p(work), _p(llrc), _p(count), _p(blocks), _p(L), _p(scratch),
                                  scratch.numel(), _stream(stream)), "lrq64_index_build")


def lr_leftmost64(llrc, blocks, total, seg_off, nseg, out, scratch, stream=None):
    _check(_lib.lrq64_lr_leftmost(_p(llrc), _p(blocks), total, _p(seg_off), _nseg(seg_off, nseg),
                                  _p(out), _p(scratch), scratch.numel(), _stream(stream)),
           "lrq64_lr_leftmost")


def lr_all_count64(llrc, blocks, total, seg_off, nseg, scratch, stream=None, want_total=True):
    out = C.c_int64(-1)
    _check(_lib.lrq64_lr_all_count(_p(llrc), _p(blocks), total, _p(seg_off),
                                   _nseg(seg_off, nseg), C.byref(out) if want_total else None,
                                   _p(scratch), scratch.numel(), _stream(stream)),
           "lrq64_lr_all_count")
    return int(out.value)


def lr_all64(llrc, blocks, total, seg_off, nseg, offsets, recs, capacity, scratch, stream=None,
             want_total=True):
    out = C.c_int64(-1)
    _check(_lib.lrq64_lr_all(_p(llrc), _p(blocks), total, _p(seg_off), _nseg(seg_off, nseg),
                             _p(offsets), _p(recs), capacity, C.byref(out) if want_total else None,
                             _p(scratch), scratch.numel(), _stream(stream)), "lrq64_lr_all")
    return int(out.value)


def lr_both64(llrc, blocks, total, seg_off, nseg, out, offsets, recs, capacity, scratch,
              stream=None, want_total=True):
    tot = C.c_int64(-1)
    _check(_lib.lrq64_lr_both(_p(llrc), _p(blocks), total, _p(seg_off), _nseg(seg_off, nseg),
                              _p(out), _p(offsets), _p(recs), capacity,
                              C.byref(tot) if want_total else None, _p(scratch), scratch.numel(),
                              _stream(stream)), "lrq64_lr_both")
    return int(tot.value)


def query_positions64(llrc, blocks, n, pos, m, out, scratch, stream=None, mode=LEFTMOST,
                      offsets=None, recs=None, capacity=0, want_total=True):
    """Point queries on one string with int64 positions (pos: int64 tensor)."""
    tot = C.c_int64(-1)
    _check(_lib.lrq64_query_positions(_p(llrc), _p(blocks), n, _p(pos), m, mode, _p(out),
                                      _p(offsets), _p(recs), capacity,
                                      C.byref(tot) if (want_total and mode == ALL) else None,
                                      _p(scratch), scratch.numel(), _stream(stream)),
           "lrq64_query_positions")
    return int(tot.value)


NOALLOC_MAX_QUERIES = 1 << 24


def query_multi_noalloc(refs, nrefs, sid, pos, m, out, stream=None, mode=LEFTMOST, offsets=None,
                        recs=None, capacity=0, want_total=True, want_errors=True):
    """lrq_query_multi without a scratch buffer (the library's own device
    array holds its counters).  Returns (record total or -1, error bits of
    this call or -1 without want_errors)."""
    tot = C.c_int64(-1)
    errs = C.c_uint32(0)
    _check(_lib.lrq_query_multi_noalloc(_p(refs), nrefs, _p(sid), _p(pos), m, mode, _p(out),
                                        _p(offsets), _p(recs), capacity,
                                        C.byref(tot) if (want_total and mode == ALL) else None,
                                        C.byref(errs) if want_errors else None, _stream(stream)),
           "lrq_query_multi_noalloc")
    return int(tot.value), (int(errs.value) if want_errors else -1)


class Tuning(C.Structure):
    """lrq_tuning: kernel shapes (results never depend on them)."""
    _fields_ = [("plcp_chunk", C.c_int32), ("llr_waves", C.c_int32), ("lr_tile", C.c_int32),
                ("fuse_filter", C.c_int32)]

    def as_dict(self):
        return {"plcp_chunk": self.plcp_chunk, "llr_waves": self.llr_waves, "lr_tile": self.lr_tile,
                "fuse_filter": self.fuse_filter}


TUNING_CHOICES = {"plcp_chunk": (8, 16, 32), "llr_waves": (4, 8), "lr_tile": (1024, 2048, 4096),
                  "fuse_filter": (0, 1)}


def set_tuning(plcp_chunk: int = 8, llr_waves: int = 8, lr_tile: int = 2048, fuse_filter: int = 0):
    t = Tuning(plcp_chunk, llr_waves, lr_tile, fuse_filter)
    _check(_lib.lrq_set_tuning(C.byref(t)), "lrq_set_tuning")


def get_tuning() -> dict:
    t = Tuning()
    _check(_lib.lrq_get_tuning(C.byref(t)), "lrq_get_tuning")
    return t.as_dict()


def timing_start(max_records: int):
    """Record HIP events around the next max_records kernel launches."""
    _check(_lib.lrq_timing_start(max_records), "lrq_timing_start")


def timing_only(kernel: str = None):
    """Record only launches of `kernel` (None: every launch)."""
    _check(_lib.lrq_timing_only(kernel.encode() if kernel else None), "lrq_timing_only")


def timing_collect(cap: int = 1 << 20):
    """[(kernel name, ms)] for the launches recorded since timing_start."""
    names = (C.c_char_p * cap)()
    ms = (C.c_float * cap)()
    cnt = C.c_int32()
    _check(_lib.lrq_timing_collect(cap, names, ms, C.byref(cnt)), "lrq_timing_collect")
    return [(names[i].decode(), float(ms[i])) for i in range(min(cnt.value, cap))]


# ------------------------------------------------------------ convenience --

class Index:
    """Device buffers and build of one string (seg_off None) or one batch.

    text: uint8 CUDA tensor; sa: int32 CUDA tensor (segment-local values), or
    int64 for the 64-bit calls (lrq64_, chosen by the SA's dtype);
    seg_off: int64 CUDA tensor of nseg+1 offsets, or None.  After
    construction ``llrc[:count]`` and ``blocks`` hold the compact index
    (global positions) and, with keep_L, ``L`` the raw LLR lengths.
    """

    def __init__(self, text, sa, seg_off=None, keep_L: bool = False, stream=None,
                 build: bool = True):
        import torch
        self.dev = text.device
        self.total = int(text.numel())
        self.seg_off = seg_off
        self.nseg = _nseg(seg_off, None)
        self.text, self.sa = text, sa
        self.stream = stream
        self.wide = sa.dtype == torch.int64
        self.dtype = torch.int64 if self.wide else torch.int32
        t = max(self.total, 1)
        self.work = torch.empty(2 * t, dtype=self.dtype, device=self.dev)
        self.llrc = torch.empty((t, 2), dtype=self.dtype, device=self.dev)
        self.count_t = torch.zeros(1, dtype=torch.int64, device=self.dev)
        self.blocks = torch.zeros(block_entries(self.total), dtype=torch.int64, device=self.dev)
        self.L = torch.empty(t, dtype=self.dtype, device=self.dev) if keep_L else None
        nbytes = (scratch_bytes64 if self.wide else scratch_bytes)(self.total, self.nseg)
        self.scratch = torch.zeros(nbytes, dtype=torch.uint8, device=self.dev)
        if build:
            self.build()

    def build(self):
        (index_build64 if self.wide else index_build)(
            self.text, self.sa, self.total, self.seg_off, self.nseg, self.work, self.llrc,
            self.count_t, self.blocks, self.L, self.scratch, self.stream)

    @property
    def count(self) -> int:
        return int(self.count_t.item())

    def compact(self):
        return self.llrc[: self.count]

    def leftmost(self, out=None):
        import torch
        if out is None:
            out = torch.empty((max(self.total, 1), 2), dtype=self.dtype, device=self.dev)
        (lr_leftmost64 if self.wide else lr_leftmost)(self.llrc, self.blocks, self.total,
                                                      self.seg_off, self.nseg, out, self.scratch,
                                                      self.stream)
        return out[: self.total]

    def all_count(self) -> int:
        return (lr_all_count64 if self.wide else lr_all_count)(
            self.llrc, self.blocks, self.total, self.seg_off, self.nseg, self.scratch,
            self.stream)

    def all(self, capacity: Optional[int] = None):
        """CSR (offsets, records); sized by a count pass unless capacity is given."""
        import torch
        cap = self.all_count() if capacity is None else capacity
        offsets = torch.empty(self.total + 1, dtype=torch.int64, device=self.dev)
        recs = torch.empty((max(cap, 1), 2), dtype=self.dtype, device=self.dev)
        total = (lr_all64 if self.wide else lr_all)(self.llrc, self.blocks, self.total,
                                                    self.seg_off, self.nseg, offsets, recs, cap,
                                                    self.scratch, self.stream)
        return offsets, recs[:total]

    def both(self, capacity: Optional[int] = None):
        """(leftmost, offsets, records) from one lrq_lr_both pass."""
        import torch
        cap = self.all_count() if capacity is None else capacity
        out = torch.empty((max(self.total, 1), 2), dtype=self.dtype, device=self.dev)
        offsets = torch.empty(self.total + 1, dtype=torch.int64, device=self.dev)
        recs = torch.empty((max(cap, 1), 2), dtype=self.dtype, device=self.dev)
        total = (lr_both64 if self.wide else lr_both)(self.llrc, self.blocks, self.total,
                                                      self.seg_off, self.nseg, out, offsets, recs,
                                                      cap, self.scratch, self.stream)
        return out[: self.total], offsets, recs[:total]

    def query(self, pos, mode: int = LEFTMOST, capacity: Optional[int] = None):
        """Point queries at the positions of the int32 tensor `pos` (int64 for
        a 64-bit index).  Leftmost mode: the (m, 2) records.  All mode:
        (leftmost records, CSR offsets, records); the record buffer starts at
        `capacity` (default 2 per query) and is enlarged once if the records
        do not fit."""
        import torch
        qfn = query_positions64 if self.wide else query_positions
        sfn = scratch_bytes64 if self.wide else scratch_bytes
        m = int(pos.numel())
        out = torch.empty((max(m, 1), 2), dtype=self.dtype, device=self.dev)
        if mode == LEFTMOST:
            qfn(self.llrc, self.blocks, self.total, pos, m, out, self.scratch, self.stream)
            return out[:m]
        scratch = self.scratch
        if sfn(max(self.total, m)) > scratch.numel():
            scratch = torch.zeros(sfn(max(self.total, m)), dtype=torch.uint8, device=self.dev)
        offsets = torch.empty(m + 1, dtype=torch.int64, device=self.dev)
        cap = 2 * m if capacity is None else capacity
        for attempt in range(2):
            recs = torch.empty((max(cap, 1), 2), dtype=self.dtype, device=self.dev)
            try:
                tot = qfn(self.llrc, self.blocks, self.total, pos, m, out, scratch, self.stream,
                          mode=ALL, offsets=offsets, recs=recs, capacity=cap)
                break
            except LrqError as e:
                if e.status != -3 or attempt:
                    raise
                # the short buffer flagged its overflow in the error word
                errs = read_errors(scratch, self.stream)
                if errs & ~ERR_CAPACITY:
                    raise LrqError(-6, "point queries", "device error bits %d" % errs)
                cap = int(offsets[m].item())
        if scratch is not self.scratch:
            errs = read_errors(scratch, self.stream)
            if errs:
                raise LrqError(-6, "point queries", "device error bits %d" % errs)
        return out[:m], offsets, recs[:tot]

    def errors(self) -> int:
        return read_errors(self.scratch, self.stream)
