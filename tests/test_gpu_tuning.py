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


def test_launch_timing_records_the_selected_kernel_only():
    """lrq_timing_start / lrq_timing_only / lrq_timing_collect: every launch,
    or only the launches of one kernel, each with a positive duration."""
    import torch
    from paper_1501_06663_amd import lrq
    text_np = workloads.dna_like(1 << 16, 2)
    dev = torch.device("cuda:0")
    idx = lrq.Index(torch.from_numpy(text_np).to(dev),
                    torch.from_numpy(lrq.build_sa_host(text_np)).to(dev), build=False)
    lrq.timing_start(1000)
    idx.build()
    allk = lrq.timing_collect()
    names = [n.split("<")[0] for n, _ in allk]
    assert "rank_scatter_kernel" in names and "llr_filter_l_kernel" in names
    assert all(ms > 0 for _, ms in allk)
    lrq.timing_only("rank_scatter_kernel")
    lrq.timing_start(1000)
    idx.build()
    idx.build()
    only = lrq.timing_collect()
    lrq.timing_only(None)
    assert [n for n, _ in only] == ["rank_scatter_kernel"] * 2
    assert idx.errors() == 0
