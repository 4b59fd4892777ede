"""Clip sets without stored FP64 spectra (CA_CLIPS_NO_FP64).

The FP64 re-decision then computes the FP64 spectra of just the clips its
groups and full-surface pairs need; every output must equal the oracle's and
the stored-FP64 set's.  This is what lets the 2M-clip scale workload (128 x
128, template densities 0.1-0.6, window +-16) stay resident on one GPU: FP16
spectra, bits and tables only."""
import numpy as np
import pytest

import clipgen
from oracle import cover

from test_gpu_parity import WORKERS, c128_subset, check_cosine, check_edge, pairs_for, periodic_set, say, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2512_13133_amd as ca
    c = ca.Context(0)
    yield c


def _sorted_pairs(cs, n, seed):
    rep, mem = pairs_for(cs, n, seed=seed)
    o = np.lexsort((mem, rep))
    return rep[o], mem[o]


@pytest.mark.parametrize("fp32", [False, True])
def test_no_fp64_c128_matches_oracle_and_stored(ctx, fp32):
    cs = c128_subset(200, seed=2)
    rep, mem = _sorted_pairs(cs, 3000, 2)
    say(f"[no-fp64] c128 pairs={rep.size} fp32={fp32}")
    h = ctx.clips(cs, fp32=fp32)
    hn = ctx.clips(cs, fp32=fp32, fp64=False)
    a = to_np(ctx.align_pairs(h, rep, mem, "cosine", (19, 20), "mixed"))
    ctx.reset_stats()
    b = to_np(ctx.align_pairs(hn, rep, mem, "cosine", (19, 20), "mixed"))
    st = ctx.stats()
    for k in a:
        assert (a[k] == b[k]).all(), k
    ref = cover.align_pairs_cosine(cs, rep, mem, 19, 20, workers=WORKERS)
    check_cosine(b, ref, rep, mem, "c128/no-fp64")
    say(f"[no-fp64] re-decided {st['pairs_rescored']} pairs, {st['groups_exact']} groups in FP64")
    assert st["pairs_rescored"] > 0
    if fp32:
        # the plain FP32 path re-decides through the same on-demand pass
        c = to_np(ctx.align_pairs(hn, rep, mem, "cosine", (19, 20), "fp32"))
        check_cosine(c, ref, rep, mem, "c128/no-fp64/fp32")
    h.close()
    hn.close()


@pytest.mark.parametrize("fp32", [False, True])
def test_no_fp64_periodic_ties(ctx, fp32):
    """Exactly tied peaks 8 rows apart: groups and full-surface pairs both go
    through the on-demand FP64 spectra."""
    cs = periodic_set(48, seed=5)
    rep, mem = _sorted_pairs(cs, None, 5)
    h = ctx.clips(cs, fp32=fp32, fp64=False)
    ctx.reset_stats()
    got = to_np(ctx.align_pairs(h, rep, mem, "cosine", (1, 2), "mixed"))
    st = ctx.stats()
    ref = cover.align_pairs_cosine(cs, rep, mem, 1, 2, workers=WORKERS)
    check_cosine(got, ref, rep, mem, "periodic/no-fp64")
    say(f"[no-fp64] periodic pairs={rep.size}: {st['groups_exact']} groups, {st['pairs_full_fp64']} full surfaces")
    assert (got["flags"] & 3).any()
    h.close()


def test_no_fp64_refusals(ctx):
    import paper_2512_13133_amd as ca
    cs = c128_subset(16, seed=4)
    h = ctx.clips(cs, fp64=False)
    for path in ("fp64", "auto"):
        with pytest.raises(ca.ClipAlignError) as e:
            ctx.align_pairs(h, [0], [1], "cosine", (19, 20), path)
        assert e.value.status == ca.CA_EUNSUPPORTED, path
    with pytest.raises(ca.ClipAlignError) as e:
        ctx.spectrum(h, 0, 128, 64)
    assert e.value.status == ca.CA_ESTATE
    h.close()
    small = clipgen.small(n_clips=4)  # 64 x 64
    with pytest.raises(ca.ClipAlignError) as e:
        ctx.clips(small, fp64=False)
    assert e.value.status == ca.CA_EUNSUPPORTED


def test_zz_scale_store_two_million_clips(ctx):
    """The scale workload at full size: 2,000,000 clips of 128 x 128 from
    20,000 templates with union densities uniform in 0.1-0.6, window +-16,
    resident on one GPU without FP64 spectra, with polygon contours.  Sampled
    pairs (a same-template partner and a uniform partner for each of 400
    clips) through the mixed cosine path, the edge track and the edge track
    over full boundary edges equal the oracle."""
    cs = clipgen.dense()
    say(f"[scale] clips={cs.n} rects={cs.rects.shape[0]}")
    h = ctx.clips(cs, fp64=False, contours=True)
    rng = np.random.default_rng(44)
    order = np.argsort(cs.template, kind="stable")
    tsorted = cs.template[order]
    anchors = rng.choice(cs.n, 400, replace=False)
    rep, mem, kind = [], [], []
    for a in anchors:
        lo, hi = np.searchsorted(tsorted, cs.template[a]), np.searchsorted(tsorted, cs.template[a], side="right")
        same = order[lo:hi]
        same = same[same != a]
        rep += [a, a]
        mem += [int(rng.choice(same)), int(rng.integers(0, cs.n))]
        kind += [0, 1]
    rep, mem, kind = np.array(rep, np.int64), np.array(mem, np.int64), np.array(kind)
    keep = rep != mem
    rep, mem, kind = rep[keep], mem[keep], kind[keep]
    ctx.reset_stats()
    got_c = to_np(ctx.align_pairs(h, rep, mem, "cosine", (19, 20), "mixed"))
    st = ctx.stats()
    got_e = to_np(ctx.align_pairs(h, rep, mem, "edge", 2))
    got_t = to_np(ctx.align_pairs(h, rep, mem, "contour", 2))
    # the oracle on the clips involved, pairs renumbered into that subset
    ids, inv = np.unique(np.concatenate([rep, mem]), return_inverse=True)
    sub = cs.subset(ids)
    srep, smem = inv[:rep.size], inv[rep.size:]
    ref_c = cover.align_pairs_cosine(sub, srep, smem, 19, 20, workers=WORKERS)
    check_cosine(got_c, ref_c, rep, mem, "scale/cosine")
    ref_e = cover.align_pairs_edge(sub, srep, smem, 2, workers=WORKERS)
    check_edge(got_e, ref_e, rep, mem, "scale/edge")
    ref_t = cover.align_pairs_contour(sub, srep, smem, 2, workers=WORKERS)
    check_edge(got_t, ref_t, rep, mem, "scale/contour")
    n_edges = [ctx.contours(h, int(i))["n_edges"] for i in ids[:200]]
    say(f"[scale] pairs={rep.size} cosine bits={int((got_c['bits'] > 0).sum())} edge bits={int((got_e['bits'] > 0).sum())} "
        f"contour bits={int((got_t['bits'] > 0).sum())} (differing contours {int(((ref_t['E'] < 0) & ~ref_t['topo']).sum())} "
        f"directions), edges per clip {min(n_edges)}-{max(n_edges)}, re-decided {st['pairs_rescored']}")
    # jittered copies of one template align far better than unrelated clips
    best = got_c["score"].max(axis=1)
    say(f"[scale] mean best cosine: same template {best[kind == 0].mean():.3f}, uniform {best[kind == 1].mean():.3f}")
    assert best[kind == 0].mean() > best[kind == 1].mean() + 0.1
    h.close()


def test_zz_scale_clusters_two_million_clips(ctx):
    """The method end to end at full scale: cosine 19/20, K = 3 on the
    2,000,000-clip workload.  The clusters are too many for the oracle's loop,
    so their validity is checked instead: the library verifies every member at
    its center on the device (any violation is an error), the assignment is a
    partition onto representatives, and the oracle re-checks 300 sampled
    members at their centers against their representatives."""
    cs = clipgen.dense()
    h = ctx.clips(cs, fp64=False)
    ctx.reset_stats()
    g = ctx.cluster(h, "cosine", (19, 20), iterations=3, path="mixed")
    st = ctx.stats()
    rep_of = g["rep_of"]
    reps = rep_of == np.arange(cs.n)
    assert (rep_of[rep_of] == rep_of).all() and g["n_clusters"] == int(reps.sum())
    assert st["center_violations"] == 0 and st["members_verified"] == int((~reps).sum())
    members = np.flatnonzero(~reps)
    pick = np.random.default_rng(1).choice(members, size=min(300, members.size), replace=False)
    ids = np.unique(np.concatenate([pick, rep_of[pick]]))
    sub = cs.subset(ids)
    pos = {int(c): k for k, c in enumerate(ids.tolist())}
    sub_rep = np.arange(sub.n, dtype=np.int32)
    sub_shift = np.zeros((sub.n, 2), np.int16)
    for m in pick.tolist():
        sub_rep[pos[m]] = pos[int(rep_of[m])]
        sub_shift[pos[m]] = g["center_shift"][m]
    bad = cover.verify_centers(sub, sub_rep, sub_shift, "cosine", (19, 20))
    say(f"[scale] clusters K=3: {g['n_clusters']} of {cs.n} clips, {members.size} members verified on the device, "
        f"{st['pairs_survived']} candidates of {st['pairs_screened']} at the loosest threshold; "
        f"oracle re-check of {pick.size} members: {len(bad)} violations")
    assert not bad
    h.close()
