"""Host-side checks of liblrq (no GPU): exports, argument validation, and the
host suffix-array builder against the oracle's independent suffix sorts."""
import ctypes as C
import itertools

import numpy as np
import pytest

import oracle
from paper_1501_06663_amd import lrq, workloads


def test_every_header_function_is_exported():
    names = lrq.header_functions()
    assert len(names) >= 15
    lib = C.CDLL(lrq.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name


def test_version_and_status_strings():
    assert lrq.version() == 4
    assert lrq.status_str(0) == "ok"
    for s in (-1, -2, -3, -4, -5, -6):
        assert lrq.status_str(s) not in ("ok", "unknown status")


def test_scratch_sizing():
    assert lrq.scratch_bytes(0) >= 256
    small, big = lrq.scratch_bytes(1000), lrq.scratch_bytes(1 << 24)
    assert big > small
    # counters, LCP seeds (16-byte pairs, one per 128 positions at the finest
    # level) and the packed text (at most 4 bits per character)
    assert (1 << 24) // 2 <= big < (1 << 24) * 11 // 16
    # the 64-bit calls size the same layout, up to their own limit
    assert lrq.scratch_bytes64(1 << 24) == big
    assert lrq.scratch_bytes64(1 << 33) > lrq.scratch_bytes64(1 << 32)
    with pytest.raises(lrq.LrqError) as e:
        lrq.scratch_bytes64(lrq.MAX_TOTAL64 + 1)
    assert e.value.status == -2
    with pytest.raises(lrq.LrqError) as e:
        lrq.scratch_bytes(-1)
    assert e.value.status == -1
    with pytest.raises(lrq.LrqError) as e:
        lrq.scratch_bytes(lrq.MAX_TOTAL + 1)
    assert e.value.status == -2


def _raw(name, *args):
    fn = getattr(lrq._lib, name)
    rc = fn(*args)
    return rc, lrq._lib.lrq_last_error().decode()


def test_validation_happens_before_any_launch():
    """Bad arguments are rejected on the host; nothing reaches the GPU (there
    is none here)."""
    fake = C.c_void_p(256)     # never dereferenced: validation fails first
    # negative size
    rc, msg = _raw("lrq_rank_scatter", fake, -5, None, 1, fake, None, fake, 1 << 20, None)
    assert rc == -1 and "total" in msg
    # too large
    rc, _ = _raw("lrq_plcp", fake, lrq.MAX_TOTAL + 1, None, 1, fake, fake, 1 << 20, None)
    assert rc == -2
    # scratch too small
    rc, msg = _raw("lrq_llr_filter", fake, 1 << 20, None, 1, fake, fake, fake, None, fake, 16, None)
    assert rc == -4 and "scratch" in msg
    # NULL scratch
    rc, _ = _raw("lrq_lr_leftmost", fake, fake, 100, None, 1, fake, None, 1 << 20, None)
    assert rc == -1
    # nseg without offsets
    rc, _ = _raw("lrq_lr_leftmost", fake, fake, 100, None, 3, fake, fake, 1 << 20, None)
    assert rc == -1
    # misaligned scratch
    rc, msg = _raw("lrq_lr_leftmost", fake, fake, 100, None, 1, fake, C.c_void_p(257), 1 << 20, None)
    assert rc == -1 and "aligned" in msg
    # NULL output
    rc, _ = _raw("lrq_lr_leftmost", fake, fake, 100, None, 1, None, fake, 1 << 20, None)
    assert rc == -1
    # negative capacity
    rc, _ = _raw("lrq_lr_all", fake, fake, 100, None, 1, fake, fake, -1, None, fake, 1 << 20, None)
    assert rc == -1
    # misaligned CSR offsets
    rc, msg = _raw("lrq_lr_all", fake, fake, 100, None, 1, C.c_void_p(264), fake, 10, None, fake,
                   1 << 20, None)
    assert rc == -1 and "offsets" in msg
    # missing block table
    rc, _ = _raw("lrq_lr_leftmost", fake, None, 100, None, 1, fake, fake, 1 << 20, None)
    assert rc == -1
    # negative query count
    rc, _ = _raw("lrq_query_positions", fake, fake, 100, fake, -1, 0, fake, None, None, 0, None,
                 fake, 1 << 20, None)
    assert rc == -1
    # unknown mode
    rc, msg = _raw("lrq_query_positions", fake, fake, 100, fake, 10, 7, fake, None, None, 0, None,
                   fake, 1 << 20, None)
    assert rc == -1 and "mode" in msg
    # all mode without CSR offsets
    rc, msg = _raw("lrq_query_multi", fake, 1, fake, fake, 10, 1, None, None, None, 0, None,
                   fake, 1 << 20, None)
    assert rc == -1 and "offsets" in msg
    # all mode whose scratch is too small for the scan of m counts
    rc, msg = _raw("lrq_query_multi", fake, 1, fake, fake, 1 << 24, 1, None, fake, fake, 10, None,
                   fake, 4096, None)
    assert rc == -4 and "scratch" in msg
    # the allocation-free query call: too many queries, bad mode, no CSR offsets
    rc, msg = _raw("lrq_query_multi_noalloc", fake, 1, fake, fake, lrq.NOALLOC_MAX_QUERIES + 1, 0,
                   fake, None, None, 0, None, None, None)
    assert rc == -2 and "LRQ_NOALLOC_MAX_QUERIES" in msg
    rc, msg = _raw("lrq_query_multi_noalloc", fake, 1, fake, fake, 10, 7, fake, None, None, 0,
                   None, None, None)
    assert rc == -1 and "mode" in msg
    rc, msg = _raw("lrq_query_multi_noalloc", fake, 1, fake, fake, 10, 1, None, None, None, 0,
                   None, None, None)
    assert rc == -1 and "offsets" in msg
    rc, msg = _raw("lrq_query_multi_noalloc", None, 1, fake, fake, 10, 0, fake, None, None, 0,
                   None, None, None)
    assert rc == -1 and "d_refs" in msg
    # read_errors with NULL
    rc, _ = _raw("lrq_read_errors", None, None, None)
    assert rc == -1
    # empty inputs are valid no-ops that launch nothing
    rc, _ = _raw("lrq_rank_scatter", None, 0, None, 1, None, None, fake, 1 << 20, None)
    assert rc == 0
    rc, _ = _raw("lrq_query_positions", fake, fake, 10, None, 0, 0, None, None, None, 0, None,
                 fake, 1 << 20, None)
    assert rc == 0


def test_int64_calls_validate_on_the_host():
    """The 32-bit calls stop at LRQ_MAX_TOTAL; the 64-bit ones take more,
    up to LRQ64_MAX_TOTAL, and want their pair buffers 16-byte aligned."""
    fake = C.c_void_p(256)     # never dereferenced: validation fails first
    rc, _ = _raw("lrq_rank_scatter", fake, lrq.MAX_TOTAL + 1, None, 1, fake, None, fake, 1 << 40,
                 None)
    assert rc == -2
    # past the size check, stopped by the NULL suffix array
    rc, msg = _raw("lrq64_rank_scatter", None, lrq.MAX_TOTAL + 1, None, 1, fake, None, fake,
                   1 << 40, None)
    assert rc == -1 and "d_sa" in msg
    rc, msg = _raw("lrq64_plcp", fake, lrq.MAX_TOTAL64 + 1, None, 1, fake, fake, 1 << 40, None)
    assert rc == -2 and "LRQ64_MAX_TOTAL" in msg
    rc, msg = _raw("lrq64_rank_scatter", fake, 100, None, 1, C.c_void_p(264), None, fake, 1 << 20,
                   None)
    assert rc == -1 and "16-byte" in msg
    rc, msg = _raw("lrq64_lr_leftmost", C.c_void_p(264), fake, 100, None, 1, fake, fake, 1 << 20,
                   None)
    assert rc == -1 and "aligned" in msg
    rc, msg = _raw("lrq64_query_positions", fake, fake, lrq.MAX_TOTAL + 5, fake, 10, 7, fake,
                   None, None, 0, None, fake, 1 << 40, None)
    assert rc == -1 and "mode" in msg


def test_host_sa_validation():
    with pytest.raises(lrq.LrqError):
        lrq.build_sa_host_batch(np.zeros(4, np.uint8), np.array([0, 3, 2, 4]))
    with pytest.raises(lrq.LrqError):
        lrq.build_sa_host_batch(np.zeros(4, np.uint8), np.array([1, 4]))
    assert lrq.build_sa_host(np.zeros(0, np.uint8)).shape == (0,)


def test_host_sa_exhaustive_small():
    for n in range(1, 9):
        for tup in itertools.product(b"abc", repeat=n):
            s = np.frombuffer(bytes(tup), np.uint8)
            assert np.array_equal(lrq.build_sa_host(s), oracle.suffix_array(s)), bytes(tup)


@pytest.mark.parametrize("kind", ["uniform", "dna", "protein", "markov", "fib", "unary", "bytes"])
def test_host_sa_matches_oracle(kind):
    n = 20000
    s = {"uniform": lambda: workloads.uniform_dna(n, 1),
         "dna": lambda: workloads.dna_like(n, 2, 8),
         "protein": lambda: workloads.protein_like(n, 3, 8),
         "markov": lambda: workloads.markov_text(n, 4),
         "fib": lambda: workloads.fibonacci_word(n),
         "unary": lambda: np.full(n, 200, np.uint8),
         "bytes": lambda: np.random.default_rng(5).integers(0, 256, n).astype(np.uint8)}[kind]()
    method = "doubling" if kind in ("fib", "unary") else "naive"
    assert np.array_equal(lrq.build_sa_host(s), oracle.suffix_array(s, method))


def test_host_sa_batch_matches_per_segment():
    text, off = workloads.config4(seed=3, nseg=12, min_log2=1, max_log2=12)
    off = off.copy()
    # include empty and one-character segments
    text = np.concatenate([text, np.array([65], np.uint8)])
    off = np.concatenate([off, [off[-1], off[-1] + 1]])
    sa = lrq.build_sa_host_batch(text, off)
    for b in range(len(off) - 1):
        seg = text[off[b]:off[b + 1]]
        assert np.array_equal(sa[off[b]:off[b + 1]], oracle.suffix_array(seg)), b


def test_single_hip_runtime_in_process():
    """liblrq must share torch's HIP runtime: two runtimes in one process would
    make torch's stream handles foreign to the library."""
    import subprocess
    import sys
    code = ("import paper_1501_06663_amd.lrq, torch\n"
            "m = open('/proc/self/maps').read().splitlines()\n"
            "libs = {l.split()[-1] for l in m if 'libamdhip64' in l}\n"
            "print(len(libs))\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         cwd=__import__("os").path.dirname(__import__("os").path.dirname(__file__)))
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "1", out.stdout


def test_header_is_c99_and_links(tmp_path):
    """include/lrq.h compiles as plain C99 and a C program links liblrq.so."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = str(tmp_path / "c_abi_check")
    libdir = os.path.dirname(lrq.LIB_PATH)
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                           "-I" + os.path.join(root, "include"),
                           os.path.join(root, "tests", "c_abi_check.c"), "-o", exe,
                           "-L" + libdir, "-llrq", "-Wl,-rpath," + libdir])
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "c abi ok"


def test_tuning_is_per_thread_without_races(tmp_path):
    """Two threads change their kernel-shape tunings concurrently through the
    C ABI.  The program is built against the library's host-only source with
    ThreadSanitizer (g++, no GPU code on the line); a data race on the tuning
    state makes it report and fail, and each thread must read back its own
    setting."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    exe = str(tmp_path / "tsan_tuning")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-fopenmp",
                           "-I" + os.path.join(root, "include"),
                           "-I" + os.path.join(root, "paper_1501_06663_amd", "csrc"),
                           "-o", exe, os.path.join(root, "tests", "tsan_tuning.cpp"),
                           os.path.join(root, "paper_1501_06663_amd", "csrc", "lrq_host.cpp")])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert "ThreadSanitizer" not in out.stderr, out.stderr[:2000]
    assert out.returncode == 0, out.stdout + out.stderr[:2000]
    assert out.stdout.strip() == "mismatches: 0 0"
