"""Every kernel shape the autotuner may pick gives the oracle's answers, on a
single string and on a batch (results must not depend on the tuning)."""
import itertools

import numpy as np
import pytest

from gpu_common import compare, gpu_stages, oracle_view, say
from paper_1501_06663_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cases():
    text, off = workloads.config4(seed=31, nseg=20, min_log2=4, max_log2=15)
    return [("dna 300k", workloads.dna_like(300_000, 17), None),
            ("batch 20", text, off)]


def test_all_tunings_match_oracle(cases):
    from paper_1501_06663_amd import lrq
    wants = [(tag, t, o, oracle_view(t, o)) for tag, t, o in cases]
    ch = lrq.TUNING_CHOICES
    names = list(ch)
    try:
        for vals in itertools.product(*(ch[k] for k in names)):
            tu = dict(zip(names, vals))
            lrq.set_tuning(**tu)
            for tag, t, o, want in wants:
                say("case: tuning", vals, tag)
                compare(gpu_stages(t, o), want, tag="%s %s" % (tag, vals))
    finally:
        lrq.set_tuning()


def test_autotuner_picks_a_valid_tuning(tmp_path, monkeypatch):
    import torch
    from paper_1501_06663_amd import autotune, lrq
    say("case: autotune on dna 1M")
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "t.json"))
    text = workloads.dna_like(1 << 20, 2)
    dev = torch.device("cuda:0")
    idx = lrq.Index(torch.from_numpy(text).to(dev), torch.from_numpy(lrq.build_sa_host(text)).to(dev))
    want = idx.leftmost().clone()
    try:
        res = autotune.tune(lambda: (idx.build(), idx.leftmost()), key="k", reps=2)
        assert set(res["tuning"]) == set(lrq.TUNING_CHOICES)
        assert lrq.get_tuning() == res["tuning"]
        again = autotune.tune(lambda: None, key="k")
        assert again["cached"] and again["tuning"] == res["tuning"]
        idx.build()
        assert torch.equal(idx.leftmost(), want)
    finally:
        lrq.set_tuning()
