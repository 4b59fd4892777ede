"""GPU parity of the edge track over full boundary edges (CA_EDGES_CONTOUR,
paper Sec. 2.2.2 over every corresponding edge; topological-hash pre-filter of
Sec. 3.1 stage 1) against the oracle (`oracle/contour.py`).

Bar: everything is integer work, so bit-exact: the per-clip contour tables
(edge words, polygon offsets, hashes), shifts, residuals, bits and flags of
the alignment, the survivor set of the pre-filter, the cover relation, the
clusters and the center verification.
"""
import sys

import numpy as np
import pytest

import clipgen
from oracle import contour, cover, raster

pytestmark = pytest.mark.gpu

WORKERS = 8


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2512_13133_amd as ca
    c = ca.Context(0)
    yield c


def to_np(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def mixed_set(seed=7, per=(24, 16, 8)):
    """Raster sizes 64/128/256, half-windows 0..32, an empty clip and a clip
    whose content is clipped away."""
    rng = np.random.default_rng(seed)
    sets = []
    for N, cnt in zip((64, 128, 256), per):
        tpl = clipgen.make_templates(rng, 4, N, 3, 10)
        w = rng.integers(0, 33, size=cnt)
        sets.append(clipgen.make_clips(rng, tpl, N, cnt, 4, w))
    cs = clipgen.concat(sets)
    return clipgen.concat([cs, clipgen.ClipSet(np.array([0, 0, 1], np.int64), np.array([[200, 300, 0, 5]], np.int32),
                                               np.array([64, 64], np.int16), np.array([3, 5], np.int16),
                                               np.array([-1, -1], np.int32), np.zeros((2, 2), np.int16))])


def low_jitter_set(seed=3, n=64, N=64, jitter=1):
    rng = np.random.default_rng(seed)
    tpl = clipgen.make_templates(rng, 8, N, 3, 10)
    return clipgen.make_clips(rng, tpl, N, n, jitter, 4)


def many_polygon_set(seed=29, n=400):
    """128 x 128 low-density many-rectangle clips: up to about 20 polygons.
    Half of the clips only move as a whole (their contours equal their
    template's unless the window clips them), half also move each rectangle
    edge by up to 1 px."""
    rng = np.random.default_rng(seed)
    dens = rng.uniform(0.1, 0.3, size=20)
    tpl = clipgen.make_templates(rng, 20, 128, 12, 24, density=dens)
    sets = []
    for jitter in (0, 1):
        tof = np.resize(np.arange(20), n // 2)
        rng.shuffle(tof)
        sets.append(clipgen.make_clips(rng, tpl, 128, n // 2, jitter, 16, template_of=tof))
    return clipgen.concat(sets)


def shapes_set():
    """Hand-made shapes: rings (holes), two holes in one polygon, pixels that
    meet diagonally inside one polygon and across two, a comb, a clip touching
    every border, and a 256 x 256 clip of 16 wavy teeth whose boundary has more
    than 4,096 edges (no contour data)."""
    clips = [
        [(1, 9, 1, 3), (1, 9, 7, 9), (1, 3, 1, 9), (7, 9, 1, 9)],                      # ring
        [(0, 20, 0, 2), (0, 20, 10, 12), (0, 2, 0, 12), (18, 20, 0, 12), (9, 11, 0, 12)],  # two holes
        [(0, 3, 0, 1), (0, 2, 1, 2), (0, 1, 2, 4), (2, 4, 2, 3), (1, 4, 3, 4)],        # diagonal touch, one polygon
        [(0, 2, 0, 2), (2, 4, 2, 4), (4, 6, 0, 2)],                                    # diagonal touch, two polygons
        [(0, 64, 0, 1)] + [(x, x + 1, 0, 40) for x in range(0, 64, 2)],               # comb
        [(0, 64, 0, 64)],                                                              # full raster
        [(0, 64, 0, 3), (0, 3, 0, 64), (61, 64, 0, 64), (0, 64, 61, 64)],              # frame on the border
    ]
    wavy = [(0, 256, 0, 1)]
    for y in range(1, 256):
        for t in range(16):
            wavy.append((16 * t + (y % 2), 16 * t + 8 + (y % 3), y, y + 1))
    ptr, rects, N = [0], [], []
    for r in clips:
        rects += r
        ptr.append(len(rects))
        N.append(64)
    rects += wavy
    ptr.append(len(rects))
    N.append(256)
    n = len(N)
    return clipgen.ClipSet(np.array(ptr, np.int64), np.array(rects, np.int32).reshape(-1, 4),
                           np.array(N, np.int16), np.full(n, 4, np.int16), np.full(n, -1, np.int32),
                           np.zeros((n, 2), np.int16))


def expected_tables(a):
    """Oracle contour tables in the library's layout, or None."""
    lab, boxes, polys = contour.clip_polygons(a)
    if polys is None:
        return None
    words, ptr, hashes = [], [], []
    for poly in polys:
        ptr.append(len(words))
        for c in poly:
            for k, (d, u) in enumerate(c):
                words.append(u | (d << 9) | ((k == 0) << 11))
        hashes.append(contour.poly_hash(poly))
    total = len(words)
    ptr += [total] * (65 - len(ptr))
    hashes += [0] * (64 - len(hashes))
    return dict(n_edges=total, edges=np.array(words, np.uint16), poly_ptr=np.array(ptr, np.uint16),
                hashes=np.array(hashes, np.uint32))


@pytest.mark.parametrize("which", ["small", "mixed", "c128", "density", "many_polygons", "shapes"])
def test_contour_tables_match_oracle(ctx, which):
    cs = {"small": lambda: clipgen.small(n_clips=96), "mixed": mixed_set,
          "c128": lambda: clipgen.c128(n_clips=600, n_templates=40),
          "density": lambda: clipgen.dense(n_clips=600, n_templates=60),
          "many_polygons": many_polygon_set, "shapes": shapes_set}[which]()
    say(f"[contour] tables {which}: clips={cs.n}")
    h = ctx.clips(cs, contours=True)
    n_holes = n_none = 0
    for i in range(cs.n):
        got = ctx.contours(h, i)
        npoly = int(ctx.inspect(h, i, int(cs.raster_n[i]))["n_poly"][0])
        want = expected_tables(raster.clip_raster(cs, i))
        if npoly < 0 or want is None:  # the labeller's cap, or more than 4,096 edges
            assert got["n_edges"] == -1, (which, i)
            n_none += 1
            continue
        assert got["n_edges"] == want["n_edges"], (which, i, got["n_edges"], want["n_edges"])
        assert (got["edges"] == want["edges"]).all(), (which, i)
        assert (got["poly_ptr"] == want["poly_ptr"]).all(), (which, i)
        assert (got["hashes"] == want["hashes"]).all(), (which, i)
        n_holes += int(((got["edges"] >> 11) & 1).sum()) - npoly
    say(f"[contour] tables {which}: equal; holes {n_holes}, clips without contour data {n_none}")
    if which == "shapes":
        assert n_none == 1 and n_holes >= 3
    h.close()


def template_pairs(cs, n_pairs, seed):
    rng = np.random.default_rng(seed)
    by_tpl = {}
    for i, t in enumerate(cs.template.tolist()):
        by_tpl.setdefault((t, int(cs.raster_n[i])), []).append(i)
    reps, mems = [], []
    for i in rng.choice(cs.n, size=n_pairs // 2, replace=cs.n < n_pairs // 2).tolist():
        mates = [j for j in by_tpl[(int(cs.template[i]), int(cs.raster_n[i]))] if j != i]
        if mates:
            reps.append(i)
            mems.append(int(rng.choice(mates)))
    r2, m2 = clipgen.same_size_pairs(cs, rng, n_pairs - len(reps))
    return (np.concatenate([np.array(reps, np.int32), r2.astype(np.int32)]),
            np.concatenate([np.array(mems, np.int32), m2.astype(np.int32)]))


def check(got, ref, rep, mem, label):
    bad = np.flatnonzero((got["bits"] != ref["bits"]) | np.any(got["shift"] != ref["shift"], axis=(1, 2)) |
                         np.any(got["count"] != ref["E"], axis=1))
    if bad.size:
        k = bad[0]
        raise AssertionError(f"{label}: {bad.size} of {rep.size} pairs differ; first k={k} rep={rep[k]} mem={mem[k]} "
                             f"got bits={got['bits'][k]} shift={got['shift'][k].tolist()} E={got['count'][k].tolist()} "
                             f"flags={got['flags'][k]:#x} ref bits={ref['bits'][k]} shift={ref['shift'][k].tolist()} "
                             f"E={ref['E'][k].tolist()}")
    # no correspondence (including differing contours) is flagged, and only then
    for d, flag in ((0, 1 << 3), (1, 1 << 4)):
        assert (((got["flags"] & flag) != 0) == (ref["E"][:, d] < 0)).all(), label
    assert (got["score"] == 0).all()


@pytest.mark.parametrize("which", ["small", "mixed", "c128", "density", "many_polygons", "low_jitter"])
def test_contour_align_matches_oracle(ctx, which):
    if which == "small":
        cs = clipgen.small(n_clips=96)
        rep, mem = clipgen.all_pairs(cs.n)
        ts = (2,)
    elif which == "mixed":
        cs = mixed_set()
        rep, mem = clipgen.same_size_pairs(cs, np.random.default_rng(4), 1500)
        ts = (3,)
    elif which == "c128":
        cs = clipgen.c128(n_clips=2000, n_templates=40)
        rep, mem = template_pairs(cs, 3001, seed=5)
        ts = (4,)
    elif which == "density":
        cs = clipgen.dense(n_clips=2000, n_templates=200)
        rep, mem = template_pairs(cs, 2000, seed=6)
        ts = (4,)
    elif which == "many_polygons":
        cs = many_polygon_set()
        rep, mem = template_pairs(cs, 1600, seed=8)
        ts = (1,)
    else:
        cs = low_jitter_set()
        rep, mem = clipgen.all_pairs(cs.n)
        ts = (0, 1, 3)
    say(f"[contour] align {which}: clips={cs.n} pairs={rep.size}")
    h = ctx.clips(cs, contours=True)
    for t in ts:
        got = to_np(ctx.align_pairs(h, rep, mem, "contour", t))
        ref = cover.align_pairs_contour(cs, rep, mem, t, workers=WORKERS)
        check(got, ref, rep, mem, f"{which}/t={t}")
        npoly = np.array([raster.components(raster.clip_raster(cs, i))[1].shape[0] for i in range(cs.n)])
        big = int((np.maximum(npoly[rep], npoly[mem]) > 8).sum())
        say(f"[contour] align {which} t={t}: equal; set bits {int((ref['bits'] & 1).sum() + (ref['bits'] >> 1).sum())}, "
            f"differing contours {int(((ref['E'] < 0) & ~ref['topo']).sum())} directions, "
            f"pairs with > 8 polygons {big}")
        if which == "many_polygons":
            assert big > 100 and (ref["bits"][np.maximum(npoly[rep], npoly[mem]) > 8] > 0).any()
        if which == "low_jitter" and t == 3:
            assert (ref["bits"] > 0).sum() > 20
    h.close()


def test_contour_prune_matches_oracle(ctx):
    """ca_prune over contours: survivors equal the oracle's pre-filter (box
    sizes and polygon hashes), and every covering pair survives."""
    cs = clipgen.concat([low_jitter_set(), low_jitter_set(seed=5, n=48, jitter=2)])
    data = [contour.clip_polygons(raster.clip_raster(cs, i)) for i in range(cs.n)]
    rep, mem = clipgen.all_pairs(cs.n)
    h = ctx.clips(cs, contours=True)
    for t in (1, 3):
        g_rep, g_mem = (x.cpu().numpy() for x in ctx.prune(h, "contour", t))
        got = set(zip(np.minimum(g_rep, g_mem).tolist(), np.maximum(g_rep, g_mem).tolist()))
        want = {(min(a, b), max(a, b)) for a, b in zip(rep.tolist(), mem.tolist())
                if contour.pair_pass(data[a], data[b], t)}
        assert got == want, (t, len(got), len(want))
        box = ctx.prune(h, "edge", t)[0].numel()
        res = cover.align_pairs_contour(cs, rep, mem, t, workers=WORKERS)
        cov = {(min(a, b), max(a, b)) for a, b, bb in zip(rep.tolist(), mem.tolist(), res["bits"].tolist()) if bb}
        assert cov <= want
        say(f"[contour] prune t={t}: {len(got)} of {rep.size} pairs survive (box sizes alone: {box}), "
            f"{len(cov)} covering")
    h.close()


def test_contour_prune_matches_oracle_many_polygons(ctx):
    """Many-polygon clips (up to about 20 polygons), where the test of per-clip
    size extremes rejects most pairs ahead of the hash and size loops: the
    survivors over contours equal the oracle's pre-filter at 1, 3 and 6 px."""
    cs = many_polygon_set(n=300)
    data = [contour.clip_polygons(raster.clip_raster(cs, i)) for i in range(cs.n)]
    rep, mem = clipgen.all_pairs(cs.n)
    h = ctx.clips(cs, contours=True)
    for t in (1, 3, 6):
        g_rep, g_mem = (x.cpu().numpy() for x in ctx.prune(h, "contour", t))
        got = set(zip(np.minimum(g_rep, g_mem).tolist(), np.maximum(g_rep, g_mem).tolist()))
        want = {(min(a, b), max(a, b)) for a, b in zip(rep.tolist(), mem.tolist())
                if contour.pair_pass(data[a], data[b], t)}
        say(f"[contour] many-polygon prune t={t}: {len(got)} survive, oracle {len(want)} of {rep.size}")
        assert want and got == want
    h.close()


def test_contour_cover_clusters_and_centers(ctx):
    cs = clipgen.concat([low_jitter_set(), low_jitter_set(seed=5, n=48, jitter=2)])
    rep, mem = clipgen.all_pairs(cs.n)
    h = ctx.clips(cs, contours=True)
    for t in (1, 3):
        ref = cover.align_pairs_contour(cs, rep, mem, t, workers=WORKERS)
        full = cover.cover_csr(cs.n, rep, mem, ref["bits"], ref["shift"], ref["E"], np.zeros((rep.size, 2)))
        got = {k: v.cpu().numpy() for k, v in ctx.cover(h, "contour", t).items()}
        for k in ("row_ptr", "col", "shift", "value"):
            assert (got[k] == full[k]).all(), (t, k)
        for K in (1, 3):
            want = cover.cluster_edge(cs, t, K=K, rep=rep, mem=mem, res=ref, edges="contour")
            g = ctx.cluster(h, "contour", t, iterations=K)
            assert g["n_clusters"] == want["n_clusters"], (t, K)
            assert (g["rep_of"] == want["rep_of"]).all() and (g["center_shift"] == want["shift"]).all(), (t, K)
            v, _ = ctx.verify_centers(h, g["rep_of"], g["center_shift"], "contour", t)
            assert v == 0
        # a moved center: the library and the oracle flag the same clips
        rep_of, shift = g["rep_of"].copy(), g["center_shift"].copy()
        members = np.flatnonzero(rep_of != np.arange(cs.n))
        shift[members[::2], 1] += 3
        v, first = ctx.verify_centers(h, rep_of, shift, "contour", t)
        bad = cover.verify_centers(cs, rep_of, shift, "contour", t)
        assert v == len(bad) and (first == (bad[0] if bad else -1))
        say(f"[contour] t={t}: cover entries {full['col'].size}, clusters K=1/3 {want['n_clusters']}, "
            f"moved centers flagged {v} of {members[::2].size}")
    h.close()


def test_contour_noalloc_and_errors(ctx):
    import paper_2512_13133_amd as ca
    cs = clipgen.concat([low_jitter_set(n=40), shapes_set()])
    rep, mem = clipgen.same_size_pairs(cs.subset(np.arange(40)), np.random.default_rng(2), 500)
    h = ctx.clips(cs, contours=True)
    a = to_np(ctx.align_pairs(h, rep, mem, "contour", 2))
    b = to_np(ctx.align_pairs(h, rep, mem, "contour", 2, noalloc=True))
    for k in a:
        assert (a[k] == b[k]).all(), k
    # the 256 x 256 wavy clip has no contour data: pairs with it are refused
    wavy = cs.n - 1
    with pytest.raises(ca.ClipAlignError) as e:
        ctx.align_pairs(h, np.array([wavy], np.int32), np.array([wavy], np.int32), "contour", 2)
    assert e.value.status == ca.CA_EUNSUPPORTED
    h2 = ctx.clips(cs.subset(np.arange(40)))
    with pytest.raises(ca.ClipAlignError) as e:
        ctx.align_pairs(h2, rep, mem, "contour", 2)
    assert e.value.status == ca.CA_ESTATE
    h.close()
    h2.close()
