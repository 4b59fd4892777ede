"""ca_align_pairs_noalloc (no device allocation inside the library) returns
exactly what ca_align_pairs returns, call after call on the shared static
work array, through the C ABI."""
import sys

import numpy as np
import pytest

import clipgen

pytestmark = pytest.mark.gpu

KEYS = ("bits", "shift", "count", "score", "flags")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2512_13133_amd as ca
    c = ca.Context(0)
    yield c


def _same(ctx, h, rep, mem, kind, thr, path, label):
    ref = {k: v.cpu().numpy() for k, v in ctx.align_pairs(h, rep, mem, kind, thr, path).items()}
    got = {k: v.cpu().numpy() for k, v in ctx.align_pairs(h, rep, mem, kind, thr, path, noalloc=True).items()}
    for k in KEYS:
        assert (got[k] == ref[k]).all(), f"{label}: {k} differs on {int((got[k] != ref[k]).sum())} entries"
    return ref


def test_noalloc_equals_align_pairs_on_consecutive_calls(ctx):
    # 128 x 128 clips with window +-16 (the batched mixed path), several
    # templates so that covers, near ties and the FP64 re-decision occur
    cs = clipgen.c128(n_clips=400, n_templates=8).subset(np.arange(0, 400, 5))
    rep, mem = clipgen.all_pairs(cs.n)
    say(f"[noalloc] c128 subset clips={cs.n} pairs={rep.size}")
    h = ctx.clips(cs, fp32=True)
    for path in ("mixed", "fp32"):
        big = _same(ctx, h, rep, mem, "cosine", (19, 20), path, f"{path} full")
        # the second call has a smaller input: stale queue contents of the first must not leak
        small = _same(ctx, h, rep[:257], mem[:257], "cosine", (19, 20), path, f"{path} small")
        for k in KEYS:
            assert (small[k] == big[k][:257]).all(), f"{path}: {k} of the smaller call"
        say(f"[noalloc] {path}: {int((big['bits'] != 0).sum())} covering pairs, "
            f"{int((big['flags'] & 3 != 0).sum())} re-decided")
    e_big = _same(ctx, h, rep, mem, "edge", 3, "mixed", "edge full")
    e_small = _same(ctx, h, rep[:100], mem[:100], "edge", 3, "mixed", "edge small")
    assert all((e_small[k] == e_big[k][:100]).all() for k in KEYS)
    h.close()


def test_noalloc_limits_are_checked_on_the_host(ctx):
    import paper_2512_13133_amd as ca
    cs = clipgen.small(n_clips=8)
    h = ctx.clips(cs)
    rep, mem = clipgen.all_pairs(cs.n)
    # FP64 path: not offered without allocation
    with pytest.raises(ca.ClipAlignError) as e:
        ctx.align_pairs(h, rep, mem, "cosine", (19, 20), "fp64", noalloc=True)
    assert e.value.status == ca.CA_EUNSUPPORTED
    # over the maximum pair count: rejected before any device work
    import ctypes as C
    con = ca.constraint("cosine", (19, 20))
    st = ctx.lib.ca_align_pairs_noalloc(ctx.h, ctx._stream(), h.handle, C.byref(con), ca.PATHS["fp32"],
                                        ca.NOALLOC_MAX_PAIRS + 1, None, None, None, None, None, None, None)
    assert st == ca.CA_EINVAL
    h.close()
