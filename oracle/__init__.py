"""Plain CPU oracle for longest-repeat queries -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it,
and it shares no code with the GPU path: the two meet only in the seeded
input generators of ``paper_1501_06663_amd.workloads``.

This module marshals numpy arrays into ``oracle.c`` (plain C, built with gcc
into ``liboracle.so`` next to it) and strings the steps together in the
paper's order: suffix array -> Rank -> LCP (Kasai) -> Lemma 1 lengths ->
compaction -> LR walks.  Citations of the paper are in ``oracle.c``.

Parity pins: every function here is pinned by tests/test_oracle_pins.py to
values the paper prints, closed forms, brute force or invariants.  The
per-position narratives of Section 5 (threads t_10 and t_9) refer to a figure
whose image is missing; they are "parity unpinned" and no function depends
on them.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain -O2, OpenMP for the per-position loops)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = C.CDLL(_LIB_PATH)
    i64, i32 = C.c_int64, C.c_int
    lib.oracle_set_threads.argtypes = [i32]
    lib.oracle_sa_naive.argtypes = [_u8p, i64, _i32p]
    lib.oracle_sa_doubling.argtypes = [_u8p, i64, _i32p]
    lib.oracle_rank.argtypes = [_i32p, i64, _i32p]
    lib.oracle_lcp_kasai.argtypes = [_u8p, i64, _i32p, _i32p, _i32p]
    lib.oracle_llr_lengths.argtypes = [_i32p, _i32p, i64, _i32p]
    lib.oracle_llr_direct.argtypes = [_u8p, i64, _i64p, i64, _i32p]
    lib.oracle_lr_leftmost_raw.argtypes = [_i32p, i64, _i32p]
    lib.oracle_lr_all_raw.argtypes = [_i32p, i64, _i64p, C.c_void_p, i64]
    lib.oracle_lr_all_raw.restype = i64
    lib.oracle_lr_window.argtypes = [_i32p, i64, C.c_void_p, C.c_void_p, C.c_void_p, i64]
    lib.oracle_lr_window.restype = i64
    lib.oracle_compact.argtypes = [_i32p, i64, _i32p]
    lib.oracle_compact.restype = i64
    lib.oracle_lr_leftmost_compact.argtypes = [_i32p, i64, i64, _i32p]
    lib.oracle_lr_all_compact.argtypes = [_i32p, i64, i64, _i64p, C.c_void_p, i64]
    lib.oracle_lr_all_compact.restype = i64
    lib.oracle_lr_brute.argtypes = [_u8p, i64, _i64p, C.c_void_p, i64]
    lib.oracle_lr_brute.restype = i64
    _lib = lib
    return lib


def set_threads(t: int) -> int:
    """Set the OpenMP thread count of the per-position loops; returns it."""
    return int(_load().oracle_set_threads(int(t)))


def _text(s) -> np.ndarray:
    if isinstance(s, (bytes, bytearray)):
        s = np.frombuffer(bytes(s), dtype=np.uint8)
    return np.ascontiguousarray(s, dtype=np.uint8)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ----------------------------------------------------------------- stages --

def suffix_array(s, method: str = "naive") -> np.ndarray:
    """SA of ``s`` (unsigned byte order; a proper prefix sorts first)."""
    s = _text(s)
    sa = np.empty(len(s), dtype=np.int32)
    fn = {"naive": _load().oracle_sa_naive, "doubling": _load().oracle_sa_doubling}[method]
    if fn(s, len(s), sa) != 0:
        raise RuntimeError("oracle suffix sort failed")
    return sa


def rank(sa: np.ndarray) -> np.ndarray:
    sa = np.ascontiguousarray(sa, dtype=np.int32)
    r = np.empty_like(sa)
    _load().oracle_rank(sa, len(sa), r)
    return r


def lcp(s, sa: np.ndarray, rk: np.ndarray) -> np.ndarray:
    """LCP[0..n] with LCP[0] = LCP[n] = 0."""
    s = _text(s)
    out = np.empty(len(s) + 1, dtype=np.int32)
    _load().oracle_lcp_kasai(s, len(s), np.ascontiguousarray(sa, np.int32),
                             np.ascontiguousarray(rk, np.int32), out)
    return out


def llr_lengths(rk: np.ndarray, lc: np.ndarray) -> np.ndarray:
    """Lemma 1: L_i = max(LCP[Rank[i]], LCP[Rank[i]+1])."""
    rk = np.ascontiguousarray(rk, np.int32)
    out = np.empty(len(rk), dtype=np.int32)
    _load().oracle_llr_lengths(rk, np.ascontiguousarray(lc, np.int32), len(rk), out)
    return out


def llr_direct(s, idx) -> np.ndarray:
    """|LLR_i| for the given positions by comparing suffix i with every other."""
    s = _text(s)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(len(idx), dtype=np.int32)
    _load().oracle_llr_direct(s, len(s), idx, len(idx), out)
    return out


def compact(L: np.ndarray) -> np.ndarray:
    """LLRc as an (m, 2) int32 array of (start, length)."""
    L = np.ascontiguousarray(L, np.int32)
    rec = np.empty((max(len(L), 1), 2), dtype=np.int32)
    m = _load().oracle_compact(L, len(L), rec)
    return rec[:m].copy()


def lr_leftmost_raw(L: np.ndarray) -> np.ndarray:
    """Algorithm 1: (n, 2) int32 of (start, length); (-1, 0) if no LR."""
    L = np.ascontiguousarray(L, np.int32)
    out = np.empty((len(L), 2), dtype=np.int32)
    _load().oracle_lr_leftmost_raw(L, len(L), out)
    return out


def lr_all_raw(L: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Algorithm 3: CSR (offsets int64[n+1], records (total, 2) int32)."""
    L = np.ascontiguousarray(L, np.int32)
    off = np.empty(len(L) + 1, dtype=np.int64)
    total = _load().oracle_lr_all_raw(L, len(L), off, None, 0)
    rec = np.empty((max(total, 1), 2), dtype=np.int32)
    _load().oracle_lr_all_raw(L, len(L), off, _ptr(rec), total)
    return off, rec[:total]


def lr_window(L: np.ndarray, mode: str = "leftmost"):
    """Sliding-window maximum form of Algorithms 1/3 (O(n + output))."""
    L = np.ascontiguousarray(L, np.int32)
    n = len(L)
    lib = _load()
    if mode == "leftmost":
        out = np.empty((n, 2), dtype=np.int32)
        lib.oracle_lr_window(L, n, _ptr(out), None, None, 0)
        return out
    off = np.empty(n + 1, dtype=np.int64)
    total = lib.oracle_lr_window(L, n, None, _ptr(off), None, 0)
    rec = np.empty((max(total, 1), 2), dtype=np.int32)
    lib.oracle_lr_window(L, n, None, _ptr(off), _ptr(rec), total)
    return off, rec[:total]


def lr_leftmost_compact(c: np.ndarray, n: int) -> np.ndarray:
    """Algorithm 2 over LLRc (stop test read as start > k)."""
    c = np.ascontiguousarray(c, np.int32).reshape(-1, 2)
    out = np.empty((n, 2), dtype=np.int32)
    _load().oracle_lr_leftmost_compact(c if len(c) else np.zeros((1, 2), np.int32), len(c), n, out)
    return out


def lr_all_compact(c: np.ndarray, n: int) -> Tuple[np.ndarray, np.ndarray]:
    """Algorithm 4 over LLRc; CSR output."""
    c = np.ascontiguousarray(c, np.int32).reshape(-1, 2)
    cc = c if len(c) else np.zeros((1, 2), np.int32)
    off = np.empty(n + 1, dtype=np.int64)
    total = _load().oracle_lr_all_compact(cc, len(c), n, off, None, 0)
    rec = np.empty((max(total, 1), 2), dtype=np.int32)
    _load().oracle_lr_all_compact(cc, len(c), n, off, _ptr(rec), total)
    return off, rec[:total]


def lr_brute(s) -> Tuple[np.ndarray, np.ndarray]:
    """Definition 1 by substring enumeration (tiny strings only); CSR output."""
    s = _text(s)
    off = np.empty(len(s) + 1, dtype=np.int64)
    total = _load().oracle_lr_brute(s, len(s), off, None, 0)
    rec = np.empty((max(total, 1), 2), dtype=np.int32)
    _load().oracle_lr_brute(s, len(s), off, _ptr(rec), total)
    return off, rec[:total]


# --------------------------------------------------------------- pipelines --

def text_order_lcp(sa: np.ndarray, rk: np.ndarray, lc: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """(LCP[Rank[i]], LCP[Rank[i]+1]) for every i: the two lcp values of
    Lemma 1 laid out by text position."""
    rk = np.asarray(rk, np.int64)
    return lc[rk].astype(np.int32), lc[rk + 1].astype(np.int32)


def pipeline(s, sa_method: str = "naive", walks: str = "raw",
             modes=("leftmost", "all")) -> Dict[str, np.ndarray]:
    """Every intermediate and result for one string, in the paper's order.

    walks="raw" uses Algorithms 1/3; walks="window" the sliding-window form
    (for strings with very long repeats).
    """
    s = _text(s)
    sa = suffix_array(s, sa_method)
    rk = rank(sa)
    lc = lcp(s, sa, rk)
    L = llr_lengths(rk, lc)
    plcp, nlcp = text_order_lcp(sa, rk, lc)
    out = {"sa": sa, "rank": rk, "lcp": lc, "plcp": plcp, "nlcp": nlcp,
           "L": L, "llrc": compact(L)}
    if "leftmost" in modes:
        out["leftmost"] = lr_leftmost_raw(L) if walks == "raw" else lr_window(L, "leftmost")
    if "all" in modes:
        off, rec = lr_all_raw(L) if walks == "raw" else lr_window(L, "all")
        out["all_offsets"], out["all_recs"] = off, rec
    return out


def pipeline_batch(text, seg_off, **kw) -> Dict[str, np.ndarray]:
    """Independent strings laid end to end: per-segment pipelines, outputs
    concatenated in segment order.  Positions in SA, starts of records and
    LLRc starts are segment-local; CSR offsets are global."""
    text = _text(text)
    seg_off = np.asarray(seg_off, dtype=np.int64)
    parts = [pipeline(text[seg_off[b]:seg_off[b + 1]], **kw) for b in range(len(seg_off) - 1)]
    out = {}
    for key in ("sa", "rank", "plcp", "nlcp", "L", "leftmost", "llrc"):
        if parts and key in parts[0]:
            out[key] = np.concatenate([p[key] for p in parts]) if parts else np.zeros(0)
    if parts and "all_offsets" in parts[0]:
        offs, recs, base = [np.zeros(1, np.int64)], [], 0
        for p in parts:
            offs.append(p["all_offsets"][1:] + base)
            recs.append(p["all_recs"])
            base += int(p["all_offsets"][-1])
        out["all_offsets"] = np.concatenate(offs)
        out["all_recs"] = np.concatenate(recs) if recs else np.zeros((0, 2), np.int32)
    out["llrc_counts"] = np.array([len(p["llrc"]) for p in parts], dtype=np.int64)
    return out
