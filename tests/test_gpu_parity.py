"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bar: bit-exact for rasters, counts, polygon tables, shifts, overlap counts,
cover bits and cluster assignments; FP64 scores within 1e-12 absolute (both
sides divide the same integers); FP16 spectra within their rounding.
"""
import sys

import numpy as np
import pytest

import clipgen
from oracle import cosine, cover, edge, prune, raster, serve

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


def small_set(n=64):
    return clipgen.small(n_clips=n)


def mixed_set(seed=7, per=(24, 16, 8)):
    """Mixed raster sizes and windows, including full-residue windows at 64."""
    rng = np.random.default_rng(seed)
    sets = []
    for N, cnt in zip((64, 128, 256), per):
        tpl = clipgen.make_templates(rng, 4, N, 3, 10)
        w = rng.integers(0, 33, size=cnt)
        sets.append(clipgen.make_clips(rng, tpl, N, cnt, 4, w))
    cs = clipgen.concat(sets)
    # an empty clip and a clip whose content is clipped away
    cs = clipgen.concat([cs, clipgen.ClipSet(np.array([0, 0, 1], np.int64), np.array([[200, 300, 0, 5]], np.int32),
                                             np.array([64, 64], np.int16), np.array([3, 5], np.int16),
                                             np.array([-1, -1], np.int32), np.zeros((2, 2), np.int16))])
    return cs


def c128_subset(n=160, seed=3):
    cs = clipgen.c128(n_clips=2000, n_templates=40)
    idx = np.sort(np.random.default_rng(seed).choice(cs.n, size=n, replace=False))
    return cs.subset(idx)


def pairs_for(cs, n_pairs=None, seed=0):
    rep, mem = clipgen.same_size_pairs(cs, np.random.default_rng(seed), n_pairs)
    return rep, mem


def to_np(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def check_cosine(got, ref, rep, mem, label):
    bits = got["bits"]
    bad = np.flatnonzero((bits != ref["bits"]) | np.any(got["shift"] != ref["shift"], axis=(1, 2)) |
                         np.any(got["count"] != ref["c"], axis=1))
    if bad.size:
        k = bad[0]
        raise AssertionError(f"{label}: {bad.size} pairs differ; first k={k} rep={rep[k]} mem={mem[k]} "
                             f"got bits={bits[k]} shift={got['shift'][k].tolist()} c={got['count'][k].tolist()} "
                             f"ref bits={ref['bits'][k]} shift={ref['shift'][k].tolist()} c={ref['c'][k].tolist()}")
    assert np.abs(got["score"] - ref["score"]).max() <= 1e-12


def check_edge(got, ref, rep, mem, label):
    bad = np.flatnonzero((got["bits"] != ref["bits"]) | np.any(got["shift"] != ref["shift"], axis=(1, 2)) |
                         np.any(got["count"] != ref["E"], axis=1))
    if bad.size:
        k = bad[0]
        raise AssertionError(f"{label}: {bad.size} pairs differ; first k={k} rep={rep[k]} mem={mem[k]} "
                             f"got bits={got['bits'][k]} shift={got['shift'][k].tolist()} E={got['count'][k].tolist()} "
                             f"ref bits={ref['bits'][k]} shift={ref['shift'][k].tolist()} E={ref['E'][k].tolist()}")
    assert (got["score"] == 0).all()


# ------------------------------------------------------------------ a1, a2


@pytest.mark.parametrize("which", ["small", "mixed"])
def test_pack_and_spectrum_match_oracle(ctx, which):
    cs = small_set(48) if which == "small" else mixed_set()
    say(f"[pack] {which} n={cs.n}")
    h = ctx.clips(cs)
    for i in range(cs.n):
        N = int(cs.raster_n[i])
        got = ctx.inspect(h, i, N)
        a = raster.clip_raster(cs, i)
        bits = np.unpackbits(got["bits"].view(np.uint8), bitorder="little").reshape(N, N).astype(bool)
        assert (bits == a).all(), f"raster of clip {i}"
        assert got["n_pix"][0] == a.sum()
        assert (got["rowsum"] == a.sum(axis=1)).all() and (got["colsum"] == a.sum(axis=0)).all()
        lab, boxes = raster.components(a)
        assert got["n_poly"][0] == boxes.shape[0], f"polygons of clip {i}"
        P = boxes.shape[0]
        assert sorted(map(tuple, got["boxes"][:P].tolist())) == sorted(map(tuple, boxes.tolist()))
        F = cosine.spectrum(a)
        W = cosine.whiten(F)
        assert got["zero_bins"][0] == int((np.abs(F) <= cosine.EPS).sum()), f"zero bins of clip {i}"
        half = W[:, :N // 2 + 1]
        sp = got["spec16"][..., 0] + 1j * got["spec16"][..., 1]
        assert np.abs(sp.real - half.real).max() <= 2.0 ** -11 + 1e-7
        assert np.abs(sp.imag - half.imag).max() <= 2.0 ** -11 + 1e-7
        assert ((sp == 0) == (half == 0)).all()
    h.close()


def _labeller_set():
    """Shapes that stress the parallel labeller: U and comb shapes whose arms
    join far below their first rows, a spiral, diagonal neighbours (separate
    under 4-connectivity), a checkerboard beyond the 64-polygon cap, random
    dense rasters, an empty and a full raster; sizes 64, 128 and 256."""
    rng = np.random.default_rng(17)
    clips = []
    def add(rects, N=128):
        clips.append((np.array(rects, np.int32).reshape(-1, 4), N))
    add([(10, 14, 10, 100), (40, 44, 10, 100), (10, 44, 96, 100)])             # U
    add([(x, x + 2, 5, 120) for x in range(4, 120, 6)] + [(4, 120, 118, 122)])  # comb joined at the bottom
    add([(10, 110, 10, 12), (108, 110, 10, 110), (20, 110, 108, 110), (20, 22, 30, 110),
         (20, 90, 30, 32), (88, 90, 30, 90), (40, 90, 88, 90), (40, 42, 50, 90)])  # spiral
    add([(x, x + 1, x, x + 1) for x in range(0, 60, 1)])                          # diagonal: 60 polygons
    add([(x, x + 1, y, y + 1) for x in range(0, 24, 2) for y in range(0, 24, 2)])  # 144 polygons: over the cap
    add([(0, 128, 0, 128)])
    add([], 64)
    for N in (64, 128, 256):
        for _ in range(3):
            m = int(rng.integers(20, 60))
            x0 = rng.integers(0, N, m); y0 = rng.integers(0, N, m)
            add(np.stack([x0, x0 + rng.integers(1, 12, m), y0, y0 + rng.integers(1, 12, m)], 1), N)
    ptr = np.cumsum([0] + [c[0].shape[0] for c in clips]).astype(np.int64)
    rects = np.concatenate([c[0] for c in clips]).astype(np.int32)
    n = len(clips)
    return clipgen.ClipSet(ptr, rects, np.array([c[1] for c in clips], np.int16), np.full(n, 4, np.int16),
                           np.full(n, -1, np.int32), np.zeros((n, 2), np.int16))


def test_labeller_matches_oracle_components(ctx):
    """Polygon counts (or -1 past the 64-polygon cap) and polygon boxes equal
    the oracle's 4-connected components on shapes whose runs merge late."""
    cs = _labeller_set()
    h = ctx.clips(cs)
    for i in range(cs.n):
        N = int(cs.raster_n[i])
        got = ctx.inspect(h, i, N)
        lab, boxes = raster.components(raster.clip_raster(cs, i))
        P = boxes.shape[0]
        if P > 64:
            assert got["n_poly"][0] == -1, f"clip {i}: {P} polygons"
            continue
        assert got["n_poly"][0] == P, f"polygons of clip {i}"
        assert sorted(map(tuple, got["boxes"][:P].tolist())) == sorted(map(tuple, boxes.tolist())), f"clip {i}"
    h.close()


def test_stored_spectra_all_precisions(ctx):
    """The FP64, FP32 and FP16 copies of every clip's whitened half-spectrum
    equal the oracle's FP64 one to their rounding (FP64: 1e-10, room for the
    two FFTs' rounding divided by |F| >= 1e-2): 128 x 128 clips through the
    fused one-workgroup transform, 64 and 256 through the two-pass one, with
    dense, sparse, empty and fully set rasters."""
    cs = mixed_set(seed=11, per=(6, 10, 3))
    rng = np.random.default_rng(5)
    extra = clipgen.ClipSet(np.array([0, 0, 1, 2], np.int64),
                            np.array([[0, 128, 0, 128], [5, 6, 7, 8]], np.int32),
                            np.array([128, 128, 128], np.int16), np.array([4, 4, 4], np.int16),
                            np.array([-1, -1, -1], np.int32), np.zeros((3, 2), np.int16))
    cs = clipgen.concat([cs, extra, c128_subset(12, seed=int(rng.integers(100)))])
    h = ctx.clips(cs, fp32=True)
    for i in range(cs.n):
        N = int(cs.raster_n[i])
        W = cosine.whiten(cosine.spectrum(raster.clip_raster(cs, i)))[:, :N // 2 + 1]
        for prec, tol in ((64, 1e-10), (32, 2.0 ** -24 + 1e-10), (16, 2.0 ** -11 + 1e-7)):
            got = ctx.spectrum(h, i, N, prec)
            err = max(np.abs(got.real - W.real).max(), np.abs(got.imag - W.imag).max())
            assert err <= tol, f"clip {i} N={N} precision {prec}: error {err:.3e}"
            assert ((got == 0) == (W == 0)).all(), f"clip {i} precision {prec}: zero bins"
    h.close()


# ------------------------------------------------------------------ a4-a6 cosine


@pytest.mark.parametrize("path", ["fp64", "fp32"])
def test_cosine_small_all_pairs(ctx, path):
    cs = small_set(64)
    rep, mem = clipgen.all_pairs(cs.n)
    say(f"[cosine] small all pairs path={path} pairs={rep.size}")
    h = ctx.clips(cs, fp32=True)
    got = to_np(ctx.align_pairs(h, rep, mem, "cosine", (19, 20), path))
    ref = cover.align_pairs_cosine(cs, rep, mem, 19, 20, workers=WORKERS)
    check_cosine(got, ref, rep, mem, f"small/{path}")
    h.close()


@pytest.mark.parametrize("path", ["fp64", "fp32"])
def test_cosine_mixed_sizes_and_windows(ctx, path):
    cs = mixed_set()
    rep, mem = pairs_for(cs, 900, seed=1)
    say(f"[cosine] mixed sizes path={path} pairs={rep.size}")
    h = ctx.clips(cs, fp32=True)
    got = to_np(ctx.align_pairs(h, rep, mem, "cosine", (97, 100), path))
    ref = cover.align_pairs_cosine(cs, rep, mem, 97, 100, workers=WORKERS)
    check_cosine(got, ref, rep, mem, f"mixed/{path}")
    empty = (got["flags"] & 4) != 0
    assert empty.any()
    h.close()


def test_cosine_auto_buckets(ctx, tmp_path):
    """CA_PATH_AUTO over mixed raster sizes and windows (64/128/256, half-windows
    0..32, empty clips): one call, buckets tuned on first use (each admitted
    path equal to FP64 on its sample), results in the caller's order equal to
    the oracle's; the tuning table survives a save/load round trip."""
    cs = mixed_set()
    rep, mem = pairs_for(cs, 1200, seed=8)
    perm = np.random.default_rng(8).permutation(rep.size)  # buckets interleaved in the input
    rep, mem = rep[perm], mem[perm]
    h = ctx.clips(cs, fp32=True)
    ctx.autotune_clear()
    got = to_np(ctx.align_pairs(h, rep, mem, "cosine", (97, 100), "auto"))
    ref = cover.align_pairs_cosine(cs, rep, mem, 97, 100, workers=WORKERS)
    check_cosine(got, ref, rep, mem, "mixed/auto")
    report = ctx.autotune_report()
    say("[auto]\n" + report)
    lines = [ln for ln in report.splitlines() if ln]
    sizes = {int(ln.split()[0][2:]) for ln in lines}
    assert sizes == {64, 128, 256}
    f = tmp_path / "tune.txt"
    ctx.autotune_save(f)
    ctx.autotune_clear()
    assert ctx.autotune_report() == ""
    ctx.autotune_load(f)
    assert ctx.autotune_report() == report
    again = to_np(ctx.align_pairs(h, rep, mem, "cosine", (97, 100), "auto"))
    check_cosine(again, ref, rep, mem, "mixed/auto/loaded")
    h.close()


def test_cosine_auto_c128_picks_mfma(ctx):
    """On 128 x 128 pairs with half-window 16 the tuner admits and picks the
    batched MFMA path (it is exact after the re-decision and fastest)."""
    cs = c128_subset(200, seed=4)
    rep, mem = pairs_for(cs, 6000, seed=4)
    o = np.lexsort((mem, rep))
    rep, mem = rep[o], mem[o]
    h = ctx.clips(cs, fp32=True)
    ctx.autotune_clear()
    got = to_np(ctx.align_pairs(h, rep, mem, "cosine", (19, 20), "auto"))
    ref = cover.align_pairs_cosine(cs, rep, mem, 19, 20, workers=WORKERS)
    check_cosine(got, ref, rep, mem, "c128/auto")
    report = ctx.autotune_report()
    say("[auto]\n" + report)
    line = [ln for ln in report.splitlines() if ln.startswith("N=128 w<=16")]
    assert line and "path=mixed" in line[0], report
    h.close()


@pytest.mark.parametrize("path", ["fp32", "fp64"])
def test_cosine_c128(ctx, path):
    cs = c128_subset(160)
    rep, mem = pairs_for(cs, 1500, seed=2)
    say(f"[cosine] c128 path={path} pairs={rep.size}")
    h = ctx.clips(cs, fp32=True)
    got = to_np(ctx.align_pairs(h, rep, mem, "cosine", (19, 20), path))
    ref = cover.align_pairs_cosine(cs, rep, mem, 19, 20, workers=WORKERS)
    check_cosine(got, ref, rep, mem, f"c128/{path}")
    h.close()


# ------------------------------------------------------------------ a7 edge


@pytest.mark.parametrize("which", ["small", "mixed"])
def test_edge_track(ctx, which):
    cs = small_set(64) if which == "small" else mixed_set()
    rep, mem = (clipgen.all_pairs(cs.n) if which == "small" else pairs_for(cs, 900, seed=4))
    t = 2
    say(f"[edge] {which} pairs={rep.size}")
    h = ctx.clips(cs)
    got = to_np(ctx.align_pairs(h, rep, mem, "edge", t))
    ref = cover.align_pairs_edge(cs, rep, mem, t, workers=WORKERS)
    check_edge(got, ref, rep, mem, which)
    h.close()


# ------------------------------------------------------------------ a3 pruning


def test_edge_track_c128(ctx):
    """128 x 128 clips with one to several polygons (single-polygon fast path
    and the polygon-plane relation), in 64-pair groups with a ragged tail."""
    cs = c128_subset(160, seed=17)
    rep, mem = pairs_for(cs, 3001, seed=17)
    say(f"[edge] c128 pairs={rep.size}")
    h = ctx.clips(cs)
    got = to_np(ctx.align_pairs(h, rep, mem, "edge", 3))
    ref = cover.align_pairs_edge(cs, rep, mem, 3, workers=WORKERS)
    npoly = np.array([len(raster.components(raster.clip_raster(cs, i))[1]) for i in range(cs.n)])
    say(f"[edge] polygons per clip: {np.bincount(npoly).tolist()}")
    assert (npoly >= 2).sum() >= 10
    check_edge(got, ref, rep, mem, "c128")
    h.close()


def _edge_strata(cs, rep, mem, npoly):
    """Stratum of each pair by the larger polygon count of its clips: 1,
    2-4, 5-8 and more than 8 (the edge kernel's LDS path)."""
    mx = np.maximum(npoly[rep], npoly[mem])
    return np.select([mx <= 1, mx <= 4, mx <= 8], [0, 1, 2], 3)


def test_edge_track_stratified_by_polygon_count(ctx):
    """128 x 128 clips with up to about 20 polygons, pairs stratified by the
    larger polygon count of the pair, half same-template pairs (polygon
    correspondences and set bits) and half uniform: clips of the density
    workload (edge 2 px), and clips of low-density many-rectangle templates
    with 1 px jitter (edge 3 px), where correspondences of more than 8
    polygons occur."""
    rng = np.random.default_rng(23)
    dens = rng.uniform(0.1, 0.3, size=40)
    tpl = clipgen.make_templates(rng, 40, 128, 12, 24, density=dens)
    tof = np.resize(np.arange(40), 800)
    rng.shuffle(tof)
    sets = [("density workload", clipgen.dense(n_clips=2000, n_templates=200), 2),
            ("many polygons", clipgen.make_clips(rng, tpl, 128, 800, 1, 16, template_of=tof), 3)]
    for label, cs, t in sets:
        npoly = np.array([len(raster.components(raster.clip_raster(cs, i))[1]) for i in range(cs.n)])
        by_tpl = {}
        for i, tp in enumerate(cs.template.tolist()):
            by_tpl.setdefault(tp, []).append(i)
        reps, mems = [], []
        for i in rng.choice(cs.n, size=min(cs.n, 800), replace=False).tolist():
            mates = [j for j in by_tpl[int(cs.template[i])] if j != i]
            for j in ([int(rng.choice(mates))] if mates else []) + [int(rng.integers(0, cs.n))]:
                reps.append(i)
                mems.append(j)
        rep, mem = np.array(reps, np.int32), np.array(mems, np.int32)
        strata = _edge_strata(cs, rep, mem, npoly)
        say(f"[edge] {label}: {rep.size} pairs, per stratum {np.bincount(strata, minlength=4).tolist()}, "
            f"max polygons {npoly.max()}")
        h = ctx.clips(cs)
        got = to_np(ctx.align_pairs(h, rep, mem, "edge", t))
        ref = cover.align_pairs_edge(cs, rep, mem, t, workers=WORKERS)
        check_edge(got, ref, rep, mem, label)
        ok = [int(ref["ok"][strata == s].sum()) for s in range(4)]
        set_bits = [int((ref["bits"][strata == s] != 0).sum()) for s in range(4)]
        say(f"[edge] {label}: correspondences per stratum {ok}, set bits {set_bits}")
        assert (strata == 3).sum() >= 100
        if label == "many polygons":
            assert ok[3] > 0 and set_bits[3] > 0
        h.close()


def test_prune_is_safe_and_matches_bounds(ctx):
    cs = small_set(96)
    say(f"[prune] cosine n={cs.n}")
    h = ctx.clips(cs)
    r, m = ctx.prune(h, "cosine", (19, 20))
    got = set(zip(r.cpu().numpy().tolist(), m.cpu().numpy().tolist()))
    got_u = {(min(a, b), max(a, b)) for a, b in got}
    assert len(got_u) == len(got)
    A = raster.rasters(cs)
    want = set()
    for i in range(cs.n):
        for j in range(i + 1, cs.n):
            if prune.cosine_pair_pass(A[i], A[j], int(cs.marker_w[i]), int(cs.marker_w[j]), 19, 20):
                want.add((i, j))
    assert got_u == want
    # safety: every covering pair survives
    rep, mem = clipgen.all_pairs(cs.n)
    ref = cover.align_pairs_cosine(cs, rep, mem, 19, 20, workers=WORKERS)
    for k in np.flatnonzero(ref["bits"]):
        assert (int(rep[k]), int(mem[k])) in got_u
    say(f"[prune] edge n={cs.n}")
    r, m = ctx.prune(h, "edge", 2)
    got_e = set(zip(r.cpu().numpy().tolist(), m.cpu().numpy().tolist()))
    want_e = set()
    boxes = [raster.components(a)[1] for a in A]
    for i in range(cs.n):
        for j in range(i + 1, cs.n):
            if prune.edge_pair_pass(boxes[i], boxes[j], 2):
                want_e.add((i, j))
    assert got_e == want_e
    h.close()


def test_edge_prune_matches_b3_on_many_polygon_clips(ctx):
    """Clips of the density workload (up to 18 polygons, 6 on average), where
    the test of per-clip size extremes rejects most pairs before the polygon
    loops of B3: the survivors equal the oracle's B3 set at 1, 3 and 6 px."""
    cs = clipgen.dense(n_clips=400, n_templates=40)
    h = ctx.clips(cs)
    A = raster.rasters(cs)
    boxes = [raster.components(a)[1] for a in A]
    for t in (1, 3, 6):
        r, m = ctx.prune(h, "edge", t)
        got = set(zip(r.cpu().numpy().tolist(), m.cpu().numpy().tolist()))
        want = {(i, j) for i in range(cs.n) for j in range(i + 1, cs.n) if prune.edge_pair_pass(boxes[i], boxes[j], t)}
        say(f"[prune] edge on density clips, {t} px: {len(got)} survivors, oracle {len(want)}")
        assert want and got == want
    h.close()


# ------------------------------------------------------------------ a10 clusters


@pytest.mark.parametrize("kind,thr,K", [("cosine", (19, 20), 1), ("cosine", (19, 20), 3), ("edge", 2, 1),
                                        ("edge", 2, 3)])
def test_cluster_matches_oracle(ctx, kind, thr, K):
    cs = small_set(96)
    say(f"[cluster] {kind} K={K} n={cs.n}")
    h = ctx.clips(cs, fp32=True)
    got = ctx.cluster(h, kind, thr, iterations=K, path="fp32")
    rep, mem = clipgen.all_pairs(cs.n)
    if kind == "cosine":
        ref = cover.cluster_cosine(cs, thr[0], thr[1], K=K, rep=rep, mem=mem, workers=WORKERS)
    else:
        ref = cover.cluster_edge(cs, thr, K=K, rep=rep, mem=mem, workers=WORKERS)
    assert got["n_clusters"] == ref["n_clusters"]
    assert (got["rep_of"] == ref["rep_of"]).all()
    assert (got["center_shift"] == ref["shift"]).all()
    h.close()


# ------------------------------------------------------------------ errors


def test_error_paths(ctx):
    import paper_2512_13133_amd as ca
    cs = small_set(8)
    h = ctx.clips(cs)
    with pytest.raises(ca.ClipAlignError) as e:
        ctx.align_pairs(h, [0, 1], [1, 99], "cosine", (19, 20), "fp64")
    assert e.value.status == ca.CA_EINVAL
    with pytest.raises(ca.ClipAlignError) as e:
        ctx.align_pairs(h, [0], [1], "cosine", (19, 20), "fp32")  # no FP32 spectra kept
    assert e.value.status == ca.CA_ESTATE
    bad = clipgen.small(n_clips=2)
    bad.raster_n[:] = 100
    with pytest.raises(ca.ClipAlignError) as e:
        ctx.clips(bad)
    assert e.value.status == ca.CA_EINVAL
    tiny = ca.Context(0, hbm_budget_bytes=1 << 16)
    with pytest.raises(ca.ClipAlignError) as e:
        tiny.clips(clipgen.small(n_clips=64))
    assert e.value.status == ca.CA_ENOMEM
    h.close()


# ------------------------------------------------------------------ mixed path


def test_mixed_surface_within_band(ctx):
    """Every window value of the FP16/MFMA surface is within a quarter of the
    re-decision band of the FP64 surface (the band is beta * sqrt(K_hi) in
    units of K r), so an undecided peak is never final."""
    import paper_2512_13133_amd as ca
    cs = c128_subset(120, seed=11)
    rep, mem = pairs_for(cs, 700, seed=5)
    say(f"[surface] c128 pairs={rep.size}")
    h = ctx.clips(cs)
    got = ctx.surface(h, rep, mem).cpu().numpy().astype(np.float64)
    band = ctx.stats()["tie_band_mixed"]
    prep = cover.Prepared(cs)
    z = {}
    worst = 0.0
    for k in range(rep.size):
        i, j = int(mem[k]), int(rep[k])
        for c in (i, j):
            if c not in z:
                z[c] = int((np.abs(cosine.spectrum(prep.a(c))) <= cosine.EPS).sum())
        r, K = cosine.surface(prep.W(i), prep.W(j))
        if K == 0:
            continue
        K_hi = 128 * 128 - max(z[i], z[j])
        ax = np.arange(-16, 17) % 128
        ref = r[np.ix_(ax, ax)] * K / K_hi
        # error in units of K r, relative to sqrt(K_hi)
        worst = max(worst, float(np.abs(got[k] - ref).max()) * K_hi / np.sqrt(K_hi))
    say(f"[surface] max |mixed - fp64| / sqrt(K_hi) = {worst:.3e}  band coefficient = {band:.2e}")
    assert worst < band / 4
    h.close()


@pytest.mark.parametrize("seed,fp32", [(2, False), (9, False), (2, True)])
def test_cosine_c128_mixed(ctx, seed, fp32):
    """The mixed path equals the oracle; with FP32 spectra its re-decision
    first screens the candidate groups on them and settles most there."""
    cs = c128_subset(200, seed=seed)
    rep, mem = pairs_for(cs, 3000, seed=seed)
    # group by representative, as candidate generation emits them, with a ragged tail
    o = np.lexsort((mem, rep))
    rep, mem = rep[o], mem[o]
    say(f"[cosine] c128 path=mixed seed={seed} fp32={fp32} pairs={rep.size}")
    h = ctx.clips(cs, fp32=fp32)
    ctx.reset_stats()
    got = to_np(ctx.align_pairs(h, rep, mem, "cosine", (19, 20), "mixed"))
    ref = cover.align_pairs_cosine(cs, rep, mem, 19, 20, workers=WORKERS)
    check_cosine(got, ref, rep, mem, "c128/mixed")
    st = ctx.stats()
    say(f"[cosine] rescored {st['pairs_rescored']} of {st['pairs_aligned']} ({st['groups_exact']} in FP64), "
        f"max peak err {st['max_surface_err']:.2e}")
    assert st["pairs_rescored"] < rep.size // 5
    if fp32:
        assert st["groups_exact"] < st["pairs_rescored"] // 2
    h.close()


def test_fp32_screen_equals_fp64_redecision(ctx):
    """The FP32 screen of the re-decision changes no result: the same pairs
    through clip sets with and without FP32 spectra give identical outputs,
    flags included (2,000 clips of the benchmark generator, 120k pairs)."""
    cs = clipgen.c128(n_clips=2_000, n_templates=60)
    h64 = ctx.clips(cs)
    h32 = ctx.clips(cs, fp32=True)
    rep, mem = ctx.prune(h64, "cosine", (19, 20))
    rep, mem = rep[:120_000], mem[:120_000]
    say(f"[screen] pairs={rep.numel()}")
    ctx.reset_stats()
    a = to_np(ctx.align_pairs(h64, rep, mem, "cosine", (19, 20), "mixed"))
    st64 = ctx.stats()
    ctx.reset_stats()
    b = to_np(ctx.align_pairs(h32, rep, mem, "cosine", (19, 20), "mixed"))
    st32 = ctx.stats()
    say(f"[screen] groups {st64['groups_exact']} -> {st32['groups_exact']} in FP64")
    for k in ("bits", "shift", "count", "score", "flags"):
        assert (a[k] == b[k]).all(), k
    assert st64["groups_exact"] > 0 and st32["groups_exact"] < st64["groups_exact"]
    h64.close()
    h32.close()


def periodic_set(n, seed):
    """128 x 128 clips that repeat exactly every 8 rows (random boxes in one
    band, copied to all 16 bands), so window surfaces have exact ties at
    shifts 8 rows apart; half-windows 16 on both sides."""
    rng = np.random.default_rng(seed)
    ptr, rects = [0], []
    for _ in range(n):
        band = []
        for _ in range(rng.integers(2, 6)):
            x0 = int(rng.integers(0, 120)); w = int(rng.integers(2, 9))
            y0 = int(rng.integers(0, 7)); h = int(rng.integers(1, 8 - y0 + 1))
            band.append((x0, min(128, x0 + w), y0, y0 + h))
        for k in range(16):
            rects += [(a, b, c + 8 * k, d + 8 * k) for (a, b, c, d) in band]
        ptr.append(len(rects))
    return clipgen.ClipSet(np.array(ptr, np.int64), np.array(rects, np.int32).reshape(-1, 4),
                           np.full(n, 128, np.int16), np.full(n, 16, np.int16), np.full(n, -1, np.int32),
                           np.zeros((n, 2), np.int16))


@pytest.mark.parametrize("fp32", [False, True])
def test_mixed_exact_ties_both_directions(ctx, fp32):
    """Exactly tied peaks (periodic clips): the FP64 re-decision of a pair
    with equal windows settles both directions with the tie rule in each
    direction's own coordinates, equal to the oracle.  With FP32 spectra the
    screen must pass every exactly tied group on to FP64."""
    cs = periodic_set(48, seed=5)
    rep, mem = pairs_for(cs, None, seed=5)
    o = np.lexsort((mem, rep))
    rep, mem = rep[o], mem[o]
    say(f"[ties] periodic pairs={rep.size} fp32={fp32}")
    h = ctx.clips(cs, fp32=fp32)
    ctx.reset_stats()
    got = to_np(ctx.align_pairs(h, rep, mem, "cosine", (1, 2), "mixed"))
    ref = cover.align_pairs_cosine(cs, rep, mem, 1, 2, workers=WORKERS)
    check_cosine(got, ref, rep, mem, "periodic/mixed")
    assert (got["flags"] & 3).any()
    assert ctx.stats()["groups_exact"] > 0
    h.close()


def test_mixed_equals_fp32_on_full_workload(ctx):
    """At the benchmark's full size (50k clips of 128 x 128, window +-16, the
    17.2M candidate pairs that pruning keeps, the launch configuration the
    benchmark times), the batched mixed path returns exactly what the
    independent FP32 per-pair path returns, and both equal the oracle on
    sampled pairs: every pair the mixed path re-decided among the sample's
    first 400, plus 400 uniform ones.  Exact ties of symmetric dense clips live
    here and nowhere in the small sets."""
    import torch
    cs = clipgen.c128(n_clips=50_000, n_templates=1_000)
    say(f"[full] clips={cs.n}")
    h = ctx.clips(cs, fp32=True)
    rep, mem = ctx.prune(h, "cosine", (19, 20))
    say(f"[full] pairs={rep.numel()}")
    ctx.reset_stats()
    om = ctx.align_pairs(h, rep, mem, "cosine", (19, 20), "mixed")
    st = ctx.stats()
    say(f"[full] mixed re-decided {st['pairs_rescored']} pairs; max peak error / sqrt(K_hi) "
        f"{st['max_peak_err_sqrt']:.4f} against band {st['tie_band_mixed']}; FP64 check of "
        f"{st['check_pairs']} decided pairs: {st['check_changed']} changed, peak error {st['check_peak_err_sqrt']:.4f}")
    assert st["max_peak_err_sqrt"] < st["tie_band_mixed"] / 2
    assert st["check_pairs"] > 0 and st["check_changed"] == 0
    assert st["check_band_frac"] < 0.5
    of = ctx.align_pairs(h, rep, mem, "cosine", (19, 20), "fp32")
    torch.cuda.synchronize()
    diff = torch.zeros(rep.numel(), dtype=torch.bool, device=rep.device)
    for k in ("bits", "shift", "count", "score"):
        d = om[k] != of[k]
        while d.dim() > 1:
            d = d.any(dim=-1)
        diff |= d
    n_diff = int(diff.sum())
    say(f"[full] mixed vs fp32: {n_diff} pairs differ")
    resc = torch.nonzero((om["flags"] & 3) != 0).flatten()[:400]
    rng = np.random.default_rng(77)
    uni = torch.as_tensor(rng.choice(rep.numel(), 400, replace=False), device=rep.device)
    sel = torch.cat([resc, uni]).cpu().numpy()
    r_np, m_np = rep.cpu().numpy()[sel], mem.cpu().numpy()[sel]
    got = {k: v.cpu().numpy()[sel] for k, v in om.items()}
    ref = cover.align_pairs_cosine(cs, r_np, m_np, 19, 20, workers=WORKERS)
    check_cosine(got, ref, r_np, m_np, "full/mixed sample")
    assert n_diff == 0
    h.close()


def test_cosine_c128_mixed_small_windows(ctx):
    """Half-windows below 16, equal and unequal within a pair, on the batched
    MFMA path (its general window search and the reverse-direction search)."""
    import dataclasses
    cs = c128_subset(160, seed=21)
    rng = np.random.default_rng(21)
    w = rng.choice(np.array([0, 1, 5, 9, 15, 16], np.int16), size=cs.n)
    cs = dataclasses.replace(cs, marker_w=w)
    rep, mem = pairs_for(cs, 2500, seed=21)
    o = np.lexsort((mem, rep))
    rep, mem = rep[o], mem[o]
    say(f"[cosine] c128 small windows path=mixed pairs={rep.size}")
    h = ctx.clips(cs)
    got = to_np(ctx.align_pairs(h, rep, mem, "cosine", (19, 20), "mixed"))
    ref = cover.align_pairs_cosine(cs, rep, mem, 19, 20, workers=WORKERS)
    check_cosine(got, ref, rep, mem, "c128/mixed/windows")
    h.close()


def test_graph_replays_match_eager(ctx):
    """The captured mixed alignment, replayed with new pair ids each time (one
    list with out-of-range ids) and eager work between replays: every replay
    equals the eager call on the same pairs; rejected pairs carry the invalid
    flag and no result."""
    import paper_2512_13133_amd as ca
    cs = c128_subset(200, seed=12)
    h = ctx.clips(cs)
    n = 3000
    g = ctx.graph(h, n, (19, 20))
    rng = np.random.default_rng(12)
    for it in range(3):
        rep = rng.integers(0, cs.n, n).astype(np.int32)
        mem = rng.integers(0, cs.n, n).astype(np.int32)
        o = np.lexsort((mem, rep))
        rep, mem = rep[o], mem[o]
        bad = np.zeros(n, bool)
        if it == 1:
            pos = rng.choice(n, 7, replace=False)
            rep[pos[:3]] = -1
            mem[pos[3:]] = cs.n + 5
            bad[pos] = True
        g.set_pairs(rep, mem)
        g.launch()
        assert g.invalid() == int(bad.sum())
        got = to_np(g.out)
        good = ~bad
        want = to_np(ctx.align_pairs(h, rep[good], mem[good], "cosine", (19, 20), "mixed"))
        for key in ("bits", "shift", "count", "score"):
            assert np.array_equal(got[key][good], want[key]), (it, key)
        mask = ca.FLAG_INVALID
        assert np.array_equal((got["flags"][good] & ~mask), want["flags"] & ~mask)
        assert ((got["flags"][bad] & mask) != 0).all()
        assert (got["bits"][bad] == 0).all() and (got["count"][bad] == -1).all()
        say(f"[graph] replay {it}: {good.sum()} pairs equal to eager, {bad.sum()} rejected")
    g.close()
    h.close()


def test_mixed_rejects_mixed_raster_sizes(ctx):
    """CA_PATH_MIXED takes clip sets of one raster size; sets that mix sizes
    go through CA_PATH_AUTO."""
    import paper_2512_13133_amd as ca
    cs = mixed_set()
    h = ctx.clips(cs)
    with pytest.raises(ca.ClipAlignError) as e:
        ctx.align_pairs(h, [0], [1], "cosine", (19, 20), "mixed")
    assert e.value.status == ca.CA_EUNSUPPORTED
    h.close()


# ------------------------------------------------------------------ launch limits


@pytest.mark.parametrize("path,n_pairs", [("fp32", (1 << 24) + 77), ("edge", (1 << 26) + 77)])
def test_launches_beyond_grid_limit(ctx, path, n_pairs):
    """More pairs than one launch can hold (grid size in work-items < 2^32): every
    replica of a pair must get the result of its first copy."""
    import torch
    cs = c128_subset(16, seed=4)
    base_rep = np.array([0, 1, 2, 3, 4, 5, 6], np.int32)
    base_mem = np.array([8, 9, 10, 11, 12, 13, 14], np.int32)
    reps = np.resize(base_rep, n_pairs)
    mems = np.resize(base_mem, n_pairs)
    say(f"[launch] {path} pairs={n_pairs}")
    h = ctx.clips(cs, fp32=True)
    if path == "edge":
        out = ctx.align_pairs(h, reps, mems, "edge", 3)
    else:
        out = ctx.align_pairs(h, reps, mems, "cosine", (19, 20), "fp32")
    m = base_rep.size
    for key in ("bits", "shift", "count", "flags"):
        v = out[key]
        first = v[:m]
        reps_t = first.repeat((n_pairs + m - 1) // m, *([1] * (v.dim() - 1)))[:n_pairs]
        assert torch.equal(v, reps_t), key
    del out
    torch.cuda.empty_cache()
    h.close()


def _oracle_prune_chunk(args):
    cs, pairs = args[:2]
    p, q = args[2] if len(args) > 2 else (19, 20)
    A = {}
    out = []
    for i, j in pairs:
        for c in (i, j):
            if c not in A:
                A[c] = raster.clip_raster(cs, c)
        if prune.cosine_pair_pass(A[i], A[j], int(cs.marker_w[i]), int(cs.marker_w[j]), p, q):
            out.append((int(i), int(j)))
    return out


def test_prune128_matches_bounds(ctx):
    """The register-resident 128 x 128 candidate generator against the oracle's bounds."""
    import multiprocessing as mp
    cs = c128_subset(360, seed=21)
    say(f"[prune128] n={cs.n}")
    h = ctx.clips(cs)
    r, m = ctx.prune(h, "cosine", (19, 20))
    r, m = r.cpu().numpy(), m.cpu().numpy()
    got = {(min(a, b), max(a, b)) for a, b in zip(r.tolist(), m.tolist())}
    assert len(got) == r.size
    ii, jj = np.triu_indices(cs.n, 1)
    chunks = np.array_split(np.arange(ii.size), 64)
    with mp.get_context("fork").Pool(WORKERS) as pool:
        res = pool.map(_oracle_prune_chunk, [(cs, list(zip(ii[c], jj[c]))) for c in chunks])
    want = set(p for part in res for p in part)
    say(f"[prune128] survivors got={len(got)} want={len(want)} of {ii.size}")
    assert got == want
    # grouping: pairs come grouped by representative (the anchor), anchors in (n, id) order
    n_pix = np.array([raster.clip_raster(cs, i).sum() for i in range(cs.n)])
    keys = [(n_pix[a], a) for a in r]
    assert keys == sorted(keys)
    h.close()


def test_prune128_matches_bounds_density_clips(ctx):
    """Density-workload clips (union densities 0.1-0.6) at 93/100, the loosest
    threshold of the K = 3 schedule: the survivors of the shift-group, coarse
    and exact stages equal the oracle's B1 + B2 set."""
    import multiprocessing as mp
    cs = clipgen.dense(n_clips=360, n_templates=36)
    h = ctx.clips(cs)
    r, m = ctx.prune(h, "cosine", (93, 100))
    r, m = r.cpu().numpy(), m.cpu().numpy()
    got = {(min(a, b), max(a, b)) for a, b in zip(r.tolist(), m.tolist())}
    assert len(got) == r.size
    ii, jj = np.triu_indices(cs.n, 1)
    chunks = np.array_split(np.arange(ii.size), 64)
    with mp.get_context("fork").Pool(WORKERS) as pool:
        res = pool.map(_oracle_prune_chunk, [(cs, list(zip(ii[c], jj[c])), (93, 100)) for c in chunks])
    want = set(p for part in res for p in part)
    say(f"[prune128] density clips at 93/100: survivors got={len(got)} want={len(want)} of {ii.size}")
    assert want and got == want
    h.close()


# ------------------------------------------------------------------ a11 serving


def _serving_case(n_library=120, n_requests=4, median=14, seed=77):
    lib, reqs = clipgen.serving(seed=seed, n_library=n_library, n_requests=n_requests, median=median,
                                sigma=0.5, max_size=40)
    return lib, [cs for _, cs in reqs]


_SERVE_ORACLE = {}  # oracle answers of the n_library=300 case, shared by both parametrisations


def _oracle_best(lib, req):
    best, score, shift, _ = serve.serve_match(lib, req, 19, 20, workers=WORKERS)
    return best, score, shift


@pytest.mark.parametrize("fp32,fp64", [(False, True), (True, True), (True, False)])
def test_serving_matches_oracle_alone_and_in_mix(ctx, fp32, fp64):
    # library ranges of ~130 partners are split into 64-partner segments, so
    # the per-segment survivor counts are summed across workgroups here; with
    # an FP32 library the near-tie re-decision runs behind the FP32 screen, and
    # without FP64 spectra (library and batches) it computes the ones it needs
    import paper_2512_13133_amd as ca
    lib, reqs = _serving_case(n_library=300)
    say(f"[serve] library={lib.n} requests={[r.n for r in reqs]} fp32={fp32} fp64={fp64}")
    hlib = ctx.clips(lib, fp32=fp32, fp64=fp64)
    srv = ca.Server(ctx, hlib, (19, 20), slots=3)
    alone = []
    for r in reqs:
        rid = srv.submit(r)
        srv.wait(rid)
        alone.append(srv.poll(rid, r.n))
    ids = [srv.submit(r) for r in reqs]
    mixed = []
    for rid, r in zip(ids, reqs):
        srv.wait(rid)
        mixed.append(srv.poll(rid, r.n))
    for a, m in zip(alone, mixed):
        for key in a:
            assert (a[key] == m[key]).all(), key
    matched = 0
    for j, (r, got) in enumerate(zip(reqs, alone)):
        if j not in _SERVE_ORACLE:
            _SERVE_ORACLE[j] = _oracle_best(lib, r)
        best, score, shift = _SERVE_ORACLE[j]
        assert (got["best_rep"] == best).all()
        assert (got["matched"] == (best >= 0)).all()
        ok = best >= 0
        assert (got["shift"][ok] == shift[ok]).all()
        assert np.abs(got["score"] - score).max() <= 1e-12
        matched += int(ok.sum())
    say(f"[serve] matched {matched} of {sum(r.n for r in reqs)} clips; stats {srv.stats()}")
    srv.close()
    hlib.close()


def test_serving_admission_budget(ctx):
    import paper_2512_13133_amd as ca
    lib, reqs = _serving_case(n_library=40, n_requests=2, median=30, seed=5)
    hlib = ctx.clips(lib)
    srv = ca.Server(ctx, hlib, (19, 20), slots=1, hbm_budget_bytes=1 << 20)
    with pytest.raises(ca.ClipAlignError) as e:
        srv.submit(reqs[0])
    assert e.value.status == ca.CA_EBUSY
    srv.close()
    hlib.close()
