"""The batching-and-precision workload at full size: 200,000 clips of mixed
raster sizes (64, 128 and 256 in ratio 4:3:1), half-windows 4..32, Zipf(1.2)
candidate lists (41.3M pairs), cosine 97/100.  One autotuned call over the
whole list; sampled outputs (500 pairs per raster size) equal the oracle."""
import numpy as np
import pytest

import clipgen
from oracle import cover

from test_gpu_parity import WORKERS, check_cosine, say

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
    rng = np.random.default_rng(33)
    pick = np.concatenate([rng.choice(np.flatnonzero(cs.raster_n[rep] == N), 500, replace=False)
                           for N in (64, 128, 256)])
    got = {k: v[torch.from_numpy(pick).cuda()].cpu().numpy() for k, v in out.items()}
    ids, inv = np.unique(np.concatenate([rep[pick], mem[pick]]), return_inverse=True)
    sub = cs.subset(ids)
    ref = cover.align_pairs_cosine(sub, inv[:pick.size], inv[pick.size:], 97, 100, workers=WORKERS)
    check_cosine(got, ref, rep[pick], mem[pick], "config3/auto")
    say(f"[config3] sampled {pick.size} pairs equal the oracle; covered {int((got['bits'] > 0).sum())}")
    h.close()
