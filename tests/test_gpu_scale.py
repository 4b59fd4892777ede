"""The batching-and-precision workload at full size: 200,000 clips of mixed
raster sizes (64, 128 and 256 in ratio 4:3:1), half-windows 4..32, Zipf(1.2)
candidate lists (41.3M pairs), cosine 97/100.  One autotuned call over the
whole list; a stratified sample of its outputs (per raster size 1,000
same-template and 1,000 uniform pairs) equals the stored oracle answers of
tests/golden/workload_mixed.npz."""
import os

import numpy as np
import pytest

import clipgen
from test_gpu_parity import check_cosine, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2512_13133_amd as ca
    c = ca.Context(0)
    yield c


def test_zz_mixed_sizes_full_list_sampled(ctx):
    import time

    import torch
    cs, rep, mem = clipgen.mixed()
    say(f"[config3] clips={cs.n} pairs={rep.size}")
    h = ctx.clips(cs, fp32=True)
    ctx.autotune_clear()
    d_rep = torch.from_numpy(rep.astype(np.int32)).cuda()
    d_mem = torch.from_numpy(mem.astype(np.int32)).cuda()
    torch.cuda.synchronize()
    t = time.perf_counter()
    out = ctx.align_pairs(h, d_rep, d_mem, "cosine", (97, 100), "auto")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    say(f"[config3] auto call {dt:.2f} s ({rep.size / dt:.3e} pairs/s, tuning included)\n" + ctx.autotune_report())
    # the stored oracle answers of a stratified sample: per raster size 1,000
    # same-template pairs (most of the covering pairs) and 1,000 uniform pairs
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "workload_mixed.npz"), allow_pickle=False)
    pick = g["pick"]
    got = {k: v[torch.from_numpy(pick).cuda()].cpu().numpy() for k, v in out.items()}
    ref = {"bits": g["bits"], "shift": g["shift"], "c": g["c"], "score": g["score"]}
    check_cosine(got, ref, rep[pick], mem[pick], "config3/auto")
    say(f"[config3] stratified sample of {pick.size} pairs equals the oracle; "
        f"{int((got['bits'] > 0).sum())} with a set bit")
    h.close()
