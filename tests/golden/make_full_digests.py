"""Write tests/golden/full_digests.json: SHA-256 digests of the CPU oracle's
outputs on the full-size workloads.

    python tests/golden/make_full_digests.py [config ...]

Calls only oracle/ (and the shared input generators); nothing here touches
the GPU path.  The full-size GPU tests compute the same digests from the GPU
outputs and require equality, which gives bit-exact parity at full size
without re-running the multi-minute oracle on the GPU machine.  The text
digest guards against generator drift.

Per config: n, segments, digests of the text, the (segment-local) suffix
array, the Lemma-1 lengths L, the
compact LLR array (global starts), the leftmost records, the all-mode CSR
offsets and records, plus per-2^20-position digests of the leftmost records so
that a mismatch can be located.
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1501_06663_amd import workloads  # noqa: E402

OUT = os.path.join(HERE, "full_digests.json")
BLOCK = 1 << 20


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def digests(text, seg_off, sa_method, walks):
    o = oracle.pipeline_batch(text, seg_off, sa_method=sa_method, walks=walks)
    glob = []
    pos = 0
    for b in range(len(seg_off) - 1):
        c = o["llrc"][pos:pos + int(o["llrc_counts"][b])].copy()
        c[:, 0] += seg_off[b]
        glob.append(c)
        pos += int(o["llrc_counts"][b])
    llrc = np.concatenate(glob).astype(np.int32)
    left = o["leftmost"].astype(np.int32)
    return {
        "n": int(len(text)), "segments": int(len(seg_off) - 1),
        "text": sha(text), "sa": sha(o["sa"].astype(np.int32)), "L": sha(o["L"].astype(np.int32)),
        "llrc": sha(llrc), "llrc_count": int(len(llrc)),
        "leftmost": sha(left),
        "leftmost_blocks": [sha(left[i:i + BLOCK]) for i in range(0, len(left), BLOCK)],
        "all_offsets": sha(o["all_offsets"].astype(np.int64)),
        "all_recs": sha(o["all_recs"].astype(np.int32)), "all_total": int(len(o["all_recs"])),
    }


CONFIGS = {
    "c1": lambda: (workloads.config1(), None, "naive", "raw"),
    "c2": lambda: (workloads.config2(), None, "naive", "raw"),
    "c3a": lambda: (workloads.config3a(), None, "doubling", "window"),
    "c3b": lambda: (workloads.config3b(), None, "naive", "raw"),
    "c4": lambda: (*workloads.config4(), "naive", "raw"),
}


def main(names):
    oracle.set_threads(os.cpu_count() or 1)
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names:
        t0 = time.time()
        text, seg, sa_method, walks = CONFIGS[name]()
        if seg is None:
            seg = np.array([0, len(text)], dtype=np.int64)
        d = digests(text, seg, sa_method, walks)
        d["oracle_seconds"] = round(time.time() - t0, 1)
        data[name] = d
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
            f.write("\n")
        print(name, d["n"], d["oracle_seconds"], "s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CONFIGS))
