"""Helpers shared by the GPU tests: run every stage of the HIP path through
the C ABI and collect its intermediates, and the oracle's view of the same
input.  The two sides share only the input bytes."""
from __future__ import annotations

import sys

import numpy as np

import oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_stages(text_np, seg_off_np=None, modes=("leftmost", "all"), want_rank=True, wide=False):
    """Run rank scatter -> PLCP -> LLR filter -> LR scans on cuda:0, stage by
    stage, and return every intermediate as numpy.  With wide, every stage
    goes through the 64-bit calls (lrq64_), on the same input."""
    import torch
    from paper_1501_06663_amd import lrq
    dev = torch.device("cuda:0")
    text_np = np.ascontiguousarray(text_np, dtype=np.uint8)
    total = len(text_np)
    if seg_off_np is None:
        sa_np = lrq.build_sa_host(text_np)
        seg, nseg = None, 1
    else:
        seg_off_np = np.ascontiguousarray(seg_off_np, dtype=np.int64)
        sa_np = lrq.build_sa_host_batch(text_np, seg_off_np)
        seg = torch.from_numpy(seg_off_np).to(dev)
        nseg = len(seg_off_np) - 1
    if wide:
        P = torch.int64
        f = {"rank_scatter": lrq.rank_scatter64, "plcp": lrq.plcp64,
             "llr_filter": lrq.llr_filter64, "index_build": lrq.index_build64,
             "lr_leftmost": lrq.lr_leftmost64, "lr_all_count": lrq.lr_all_count64,
             "lr_all": lrq.lr_all64, "lr_both": lrq.lr_both64, "scratch": lrq.scratch_bytes64}
        sa_np = sa_np.astype(np.int64)
    else:
        P = torch.int32
        f = {"rank_scatter": lrq.rank_scatter, "plcp": lrq.plcp, "llr_filter": lrq.llr_filter,
             "index_build": lrq.index_build, "lr_leftmost": lrq.lr_leftmost,
             "lr_all_count": lrq.lr_all_count, "lr_all": lrq.lr_all, "lr_both": lrq.lr_both,
             "scratch": lrq.scratch_bytes}
    t = max(total, 1)
    text = torch.from_numpy(np.concatenate([text_np, np.zeros(1, np.uint8)])).to(dev)
    sa = torch.from_numpy(np.concatenate([sa_np, np.zeros(1, sa_np.dtype)])).to(dev)
    scratch = torch.zeros(f["scratch"](total, nseg), dtype=torch.uint8, device=dev)
    work = torch.full((2 * t,), -7, dtype=P, device=dev)
    rank = torch.full((t,), -7, dtype=P, device=dev) if want_rank else None
    out = {"sa": sa_np}
    f["rank_scatter"](sa, total, seg, nseg, work, rank, scratch)
    out["nbr"] = work[: 2 * total].view(-1, 2).cpu().numpy().copy()
    if rank is not None:
        out["rank"] = rank[:total].cpu().numpy()
        # without a Rank output the scatter may take its bucketed form
        w2 = torch.full((2 * t,), -7, dtype=P, device=dev)
        f["rank_scatter"](sa, total, seg, nseg, w2, None, scratch)
        out["nbr_norank"] = w2[: 2 * total].view(-1, 2).cpu().numpy()
    f["plcp"](text, total, seg, nseg, work, scratch)
    out["pn"] = work[: 2 * total].view(-1, 2).cpu().numpy().copy()
    llrc = torch.full((t, 2), -7, dtype=P, device=dev)
    count = torch.full((1,), -7, dtype=torch.int64, device=dev)
    blocks = torch.full((lrq.block_entries(total),), -7, dtype=torch.int64, device=dev)
    L = torch.full((t,), -7, dtype=P, device=dev)
    f["llr_filter"](work, total, seg, nseg, llrc, count, blocks, L, scratch)
    m = int(count.item())
    out["llrc"] = llrc[:m].cpu().numpy()
    out["blocks"] = blocks.cpu().numpy()
    out["L"] = L[:total].cpu().numpy()
    # the build entry point (rank scatter -> LCP -> filter in one call; the LCP
    # walk and the filter are one kernel or two, by tuning)
    fl = torch.full((t, 2), -7, dtype=P, device=dev)
    fc = torch.full((1,), -7, dtype=torch.int64, device=dev)
    fb = torch.full((lrq.block_entries(total),), -7, dtype=torch.int64, device=dev)
    fL = torch.full((t,), -7, dtype=P, device=dev)
    fw = torch.full((2 * t,), -7, dtype=P, device=dev)
    f["index_build"](text, sa, total, seg, nseg, fw, fl, fc, fb, fL, scratch)
    out["fused_llrc"] = fl[: int(fc.item())].cpu().numpy()
    out["fused_blocks"] = fb.cpu().numpy()
    out["fused_L"] = fL[:total].cpu().numpy()
    if "leftmost" in modes:
        res = torch.full((t, 2), -7, dtype=P, device=dev)
        f["lr_leftmost"](llrc, blocks, total, seg, nseg, res, scratch)
        out["leftmost"] = res[:total].cpu().numpy()
    if "all" in modes:
        tot = f["lr_all_count"](llrc, blocks, total, seg, nseg, scratch)
        offs = torch.full((total + 1,), -7, dtype=torch.int64, device=dev)
        recs = torch.full((max(tot, 1), 2), -7, dtype=P, device=dev)
        tot2 = f["lr_all"](llrc, blocks, total, seg, nseg, offs, recs, tot, scratch)
        assert tot2 == tot, (tot2, tot)
        out["all_offsets"] = offs.cpu().numpy()
        out["all_recs"] = recs[:tot].cpu().numpy()
    if "leftmost" in modes and "all" in modes:
        # both modes in one pass
        lres = torch.full((t, 2), -7, dtype=P, device=dev)
        offs = torch.full((total + 1,), -7, dtype=torch.int64, device=dev)
        recs = torch.full((max(tot, 1), 2), -7, dtype=P, device=dev)
        tot3 = f["lr_both"](llrc, blocks, total, seg, nseg, lres, offs, recs, tot, scratch)
        assert tot3 == tot, (tot3, tot)
        out["both_leftmost"] = lres[:total].cpu().numpy()
        out["both_offsets"] = offs.cpu().numpy()
        out["both_recs"] = recs[:tot].cpu().numpy()
    out["errors"] = lrq.read_errors(scratch)
    return out


def oracle_view(text_np, seg_off_np=None, walks="raw", sa_method="naive"):
    """The oracle's results, per segment, with the GPU path's global/local
    conventions: LLRc starts global, record starts local."""
    text_np = np.ascontiguousarray(text_np, dtype=np.uint8)
    if seg_off_np is None:
        seg_off_np = np.array([0, len(text_np)], dtype=np.int64)
    o = oracle.pipeline_batch(text_np, seg_off_np, walks=walks, sa_method=sa_method)
    n = len(text_np)
    phi = np.full((n, 2), -1, dtype=np.int32)
    llrc_glob = []
    pos = 0
    for b in range(len(seg_off_np) - 1):
        s0, s1 = int(seg_off_np[b]), int(seg_off_np[b + 1])
        sa = o["sa"][s0:s1].astype(np.int64)
        if s1 > s0:
            prev = np.concatenate([[-1], sa[:-1] + s0])
            nxt = np.concatenate([sa[1:] + s0, [-1]])
            phi[sa + s0, 0] = prev
            phi[sa + s0, 1] = nxt
        c = o["llrc"][pos:pos + int(o["llrc_counts"][b])].copy()
        c[:, 0] += s0
        llrc_glob.append(c)
        pos += int(o["llrc_counts"][b])
    o["nbr"] = phi
    o["pn"] = np.stack([o["plcp"], o["nlcp"]], axis=1) if n else np.zeros((0, 2), np.int32)
    o["llrc_global"] = np.concatenate(llrc_glob) if llrc_glob else np.zeros((0, 2), np.int32)
    # block table: entries starting before j * 1024, and their total
    starts = o["llrc_global"][:, 0].astype(np.int64)
    edges = np.arange(0, (n + 1023) // 1024 + 1, dtype=np.int64) * 1024
    o["blocks"] = np.searchsorted(starts, np.minimum(edges, n), side="left").astype(np.int64)
    o["blocks"][-1] = len(starts)
    return o


def compare(g, o, keys=("rank", "nbr", "pn", "L", "llrc", "blocks", "leftmost", "all"), tag=""):
    """Element-by-element equality; raises with the first differing index."""
    def eq(name, a, b):
        a, b = np.asarray(a), np.asarray(b)
        assert a.shape == b.shape, "%s %s: shape %s vs oracle %s" % (tag, name, a.shape, b.shape)
        if a.size and not np.array_equal(a, b):
            bad = np.argwhere(a != b)[0]
            raise AssertionError("%s %s differs at %s: gpu %s oracle %s" % (
                tag, name, bad.tolist(), a[tuple(bad[:1])].tolist(), b[tuple(bad[:1])].tolist()))
    if "nbr_norank" in g:
        eq("nbr (no rank)", g["nbr_norank"], o["nbr"])
    if "fused_llrc" in g:
        eq("fused llrc", g["fused_llrc"], o["llrc_global"])
        eq("fused blocks", g["fused_blocks"], o["blocks"])
        eq("fused L", g["fused_L"], o["L"])
    for k in keys:
        if k == "llrc":
            eq("llrc", g["llrc"], o["llrc_global"])
        elif k == "all":
            if "all_offsets" in g:
                eq("all_offsets", g["all_offsets"], o["all_offsets"])
                eq("all_recs", g["all_recs"], o["all_recs"])
            if "both_offsets" in g:
                eq("both leftmost", g["both_leftmost"], o["leftmost"])
                eq("both offsets", g["both_offsets"], o["all_offsets"])
                eq("both recs", g["both_recs"], o["all_recs"])
        elif k == "rank":
            if "rank" in g:
                eq("rank", g["rank"], o["rank"])
        elif k in g:
            eq(k, g[k], o[k])
    assert g["errors"] == 0, "%s device error bits %d" % (tag, g["errors"])
