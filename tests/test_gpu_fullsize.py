"""Full-size parity: the HIP path on the five full workloads (16M DNA-like,
4M Fibonacci, 64M Markov text, the 512-string batch, and the 64K uniform
string), in the launch configuration bench.py times, compared bit for bit
with the CPU oracle through SHA-256 digests of every output.

The digests were written by tests/golden/make_full_digests.py, which calls
only the oracle; the inputs are regenerated here from the same seeded
generators and their digest is checked first, so generator drift shows up as
its own failure."""
import hashlib
import json
import os

import numpy as np
import pytest

from gpu_common import say
from paper_1501_06663_amd import workloads

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "full_digests.json")
with open(GOLD) as f:
    DIGESTS = json.load(f)

INPUTS = {
    "c1": lambda: (workloads.config1(), None),
    "c2": lambda: (workloads.config2(), None),
    "c3a": lambda: (workloads.config3a(), None),
    "c3b": lambda: (workloads.config3b(), None),
    "c4": lambda: workloads.config4(),
}


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.mark.parametrize("name", sorted(DIGESTS))
def test_full_size_digests(name):
    import torch
    from paper_1501_06663_amd import lrq
    want = DIGESTS[name]
    say("case: full-size", name, "n=%d segments=%d" % (want["n"], want["segments"]))
    text_np, seg_np = INPUTS[name]()
    assert sha(text_np) == want["text"], "generator output changed; regenerate the digests"
    dev = torch.device("cuda:0")
    if seg_np is None:
        sa_np = lrq.build_sa_host(text_np)
        seg = None
    else:
        sa_np = lrq.build_sa_host_batch(text_np, seg_np)
        seg = torch.from_numpy(seg_np).to(dev)
    say("  host SA built; running the GPU path")
    idx = lrq.Index(torch.from_numpy(text_np).to(dev), torch.from_numpy(sa_np).to(dev), seg,
                    keep_L=True)
    m = idx.count
    assert m == want["llrc_count"]
    assert sha(idx.compact().cpu().numpy()) == want["llrc"], "compact LLR array"
    assert sha(idx.L[: idx.total].cpu().numpy()) == want["L"], "Lemma-1 lengths"
    left = idx.leftmost().cpu().numpy()
    if sha(left) != want["leftmost"]:
        blocks = [sha(left[i:i + (1 << 20)]) for i in range(0, len(left), 1 << 20)]
        bad = [i for i, (a, b) in enumerate(zip(blocks, want["leftmost_blocks"])) if a != b]
        raise AssertionError("leftmost records differ in 2^20-blocks %s" % bad[:10])
    off, recs = idx.all()
    assert int(recs.shape[0]) == want["all_total"]
    assert sha(off.cpu().numpy()) == want["all_offsets"], "all-mode offsets"
    assert sha(recs.cpu().numpy()) == want["all_recs"], "all-mode records"
    assert idx.errors() == 0
