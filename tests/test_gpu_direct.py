"""GPU parity of the direct (spatial-domain) MFMA path against the FP64 oracle.

Bar: FP16 whitened images within their rounding of the oracle's; every
window value of the low-precision surface within a quarter of the
re-decision band of the FP64 surface; shifts, overlap counts and cover bits
bit-exact and FP64 scores within 1e-12 (both sides divide the same integers).
"""
import dataclasses
import sys

import numpy as np
import pytest

import clipgen
from oracle import cosine, cover, raster

pytestmark = pytest.mark.gpu

# The direct kernel's first GPU run ended in a memory-aperture fault whose
# cause has not been identified; the library keeps the path switched off
# (CA_EUNSUPPORTED) and its GPU tests stay skipped until the cause is found.
DIRECT_OFF = pytest.mark.skip(reason="direct path switched off: unexplained GPU fault on its first run")

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


def small_window_set(N, n, seed, w_choices=(0, 1, 3, 5, 7), n_templates=6, empty=False):
    """Clips of one raster size with half-windows <= 7 from a few templates
    (so that many pairs are near matches), optionally with an empty clip."""
    rng = np.random.default_rng(seed)
    tpl = clipgen.make_templates(rng, n_templates, N, 3, 12)
    w = rng.choice(np.array(w_choices, np.int64), size=n)
    cs = clipgen.make_clips(rng, tpl, N, n, 3, w)
    if empty:
        e = clipgen.ClipSet(np.array([0, 0], np.int64), np.zeros((0, 4), np.int32), np.array([N], np.int16),
                            np.array([2], np.int16), np.array([-1], np.int32), np.zeros((1, 2), np.int16))
        cs = clipgen.concat([cs, e])
    return cs


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


def run_pairs(n, n_pairs, seed, sort):
    """Pairs of a clip set of n clips: sorted by representative (runs of
    uneven length, several tiles and a ragged tail) or in random order (runs
    of one)."""
    rng = np.random.default_rng(seed)
    rep = rng.integers(0, n, n_pairs).astype(np.int32)
    mem = rng.integers(0, n, n_pairs).astype(np.int32)
    if sort:
        o = np.lexsort((mem, rep))
        rep, mem = rep[o], mem[o]
    return rep, mem


# ------------------------------------------------------------------ a2 (image)


def test_images_match_oracle(ctx):
    """The stored image N * IDFT2(W) equals the oracle's within FP16 rounding,
    for every raster size."""
    rng = np.random.default_rng(31)
    sets = []
    for N, cnt in ((64, 6), (128, 6), (256, 3)):
        tpl = clipgen.make_templates(rng, 3, N, 3, 10)
        sets.append(clipgen.make_clips(rng, tpl, N, cnt, 4, 7))
    cs = clipgen.concat(sets)
    h = ctx.clips(cs, image=True)
    for i in range(cs.n):
        N = int(cs.raster_n[i])
        a = raster.clip_raster(cs, i)
        ref = cosine.whitened_image(cosine.whiten(cosine.spectrum(a)))
        got = ctx.image(h, i, N).astype(np.float64)
        err = np.abs(got - ref) - (2.0 ** -11 * np.abs(ref) + 1e-6)
        assert err.max() <= 0, f"clip {i} N={N}: worst excess {err.max():.3e}"
    h.close()


# ------------------------------------------------------------------ a4' (surface)


@DIRECT_OFF
@pytest.mark.parametrize("N", [64, 128, 256])
def test_direct_surface_within_band(ctx, N):
    """Every window value (|dy|, |dx| <= 7) of the FP16 direct surface is
    within a quarter of the re-decision band of the FP64 surface."""
    n = {64: 80, 128: 60, 256: 24}[N]
    cs = small_window_set(N, n, seed=40 + N)
    rep, mem = run_pairs(cs.n, {64: 600, 128: 400, 256: 120}[N], seed=N, sort=True)
    say(f"[direct surface] N={N} pairs={rep.size}")
    h = ctx.clips(cs, image=True)
    got = ctx.surface(h, rep, mem, path="direct").cpu().numpy().astype(np.float64)
    band = ctx.stats()["tie_band_direct"]
    prep = cover.Prepared(cs)
    z = {}
    worst = 0.0
    ax = np.arange(-7, 8) % N
    for k in range(rep.size):
        i, j = int(mem[k]), int(rep[k])
        for c in (i, j):
            if c not in z:
                z[c] = int((np.abs(cosine.spectrum(prep.a(c))) <= cosine.EPS).sum())
        r, K = cosine.surface(prep.W(i), prep.W(j))
        if K == 0:
            continue
        K_hi = N * N - max(z[i], z[j])
        ref = r[np.ix_(ax, ax)] * K / K_hi
        worst = max(worst, float(np.abs(got[k, 9:24, 9:24] - ref).max()))
    say(f"[direct surface] N={N} max |direct - fp64| = {worst:.3e}  band = {band:.1e}")
    assert worst < band / 4
    h.close()


# ------------------------------------------------------------------ a4'-a6 (results)


@DIRECT_OFF
@pytest.mark.parametrize("N,sort", [(64, True), (128, True), (128, False), (256, True)])
def test_direct_matches_oracle(ctx, N, sort):
    """Cover bits, shifts, counts and scores of the direct path equal the
    oracle's: windows 0..7 equal and unequal within a pair, self pairs, an
    empty clip, representative runs of every length and a ragged last tile."""
    n = {64: 90, 128: 70, 256: 24}[N]
    cs = small_window_set(N, n, seed=50 + N, empty=True)
    n_pairs = {64: 3000, 128: 2000, 256: 300}[N] + 37
    rep, mem = run_pairs(cs.n, n_pairs, seed=N + int(sort), sort=sort)
    rep[:5] = mem[:5]  # self pairs
    if sort:
        o = np.lexsort((mem, rep))
        rep, mem = rep[o], mem[o]
    say(f"[direct] N={N} sorted={sort} pairs={rep.size}")
    h = ctx.clips(cs, image=True)
    got = to_np(ctx.align_pairs(h, rep, mem, "cosine", (19, 20), "direct"))
    ref = cover.align_pairs_cosine(cs, rep, mem, 19, 20, workers=WORKERS)
    check_cosine(got, ref, rep, mem, f"direct/{N}")
    st = ctx.stats()
    say(f"[direct] N={N} rescored={st['pairs_rescored']} max_err={st['max_surface_err']:.2e}")
    h.close()


@DIRECT_OFF
def test_direct_c128_workload_windows(ctx):
    """128 x 128 clips of the benchmark generator (6-24 rectangles, jitter 4)
    with half-windows <= 7: equal to the FP64 path on thousands of pairs."""
    cs = clipgen.c128(n_clips=400, n_templates=20, w=7)
    rng = np.random.default_rng(61)
    cs = dataclasses.replace(cs, marker_w=rng.choice(np.array([3, 4, 7], np.int16), size=cs.n))
    rep, mem = run_pairs(cs.n, 6000, seed=61, sort=True)
    say(f"[direct] c128 w<=7 pairs={rep.size}")
    h = ctx.clips(cs, image=True)
    got = to_np(ctx.align_pairs(h, rep, mem, "cosine", (19, 20), "direct"))
    ref = to_np(ctx.align_pairs(h, rep, mem, "cosine", (19, 20), "fp64"))
    for key in ("bits", "shift", "count", "score"):
        assert (got[key] == ref[key]).all(), key
    sub = np.arange(0, rep.size, 7)
    oref = cover.align_pairs_cosine(cs, rep[sub], mem[sub], 19, 20, workers=WORKERS)
    check_cosine({k: v[sub] for k, v in got.items()}, oref, rep[sub], mem[sub], "direct/c128")
    h.close()


@DIRECT_OFF
def test_direct_rejects_other_shapes(ctx):
    import paper_2512_13133_amd as ca
    cs = small_window_set(64, 8, seed=3)
    h = ctx.clips(cs)  # no images
    with pytest.raises(ca.ClipAlignError) as e:
        ctx.align_pairs(h, [0], [1], "cosine", (19, 20), "direct")
    assert e.value.status == ca.CA_ESTATE
    h.close()
    wide = dataclasses.replace(cs, marker_w=np.full(cs.n, 8, np.int16))
    h = ctx.clips(wide, image=True)
    with pytest.raises(ca.ClipAlignError) as e:
        ctx.align_pairs(h, [0], [1], "cosine", (19, 20), "direct")
    assert e.value.status == ca.CA_EUNSUPPORTED
    h.close()
    two = clipgen.concat([cs, small_window_set(128, 4, seed=4)])
    h = ctx.clips(two, image=True)
    with pytest.raises(ca.ClipAlignError) as e:
        ctx.align_pairs(h, [0], [1], "cosine", (19, 20), "direct")
    assert e.value.status == ca.CA_EUNSUPPORTED
    h.close()


# ------------------------------------------------------------------ a9 (tuner)


@DIRECT_OFF
def test_auto_with_direct_candidates(ctx):
    """CA_PATH_AUTO on a set with images: the small-window buckets time the
    direct path among the admitted candidates, and the results in the
    caller's order equal the oracle's."""
    rng = np.random.default_rng(71)
    sets = []
    for N, cnt in ((64, 40), (128, 40), (256, 10)):
        tpl = clipgen.make_templates(rng, 4, N, 3, 10)
        w = rng.choice(np.array([2, 4, 6, 7, 12, 16], np.int64), size=cnt)
        sets.append(clipgen.make_clips(rng, tpl, N, cnt, 3, w))
    cs = clipgen.concat(sets)
    rep, mem = clipgen.same_size_pairs(cs, np.random.default_rng(72), 2500)
    perm = np.random.default_rng(73).permutation(rep.size)
    rep, mem = rep[perm], mem[perm]
    h = ctx.clips(cs, image=True)
    ctx.autotune_clear()
    got = to_np(ctx.align_pairs(h, rep, mem, "cosine", (97, 100), "auto"))
    ref = cover.align_pairs_cosine(cs, rep, mem, 97, 100, workers=WORKERS)
    check_cosine(got, ref, rep, mem, "auto/direct")
    report = ctx.autotune_report()
    say("[auto]\n" + report)
    small = [ln for ln in report.splitlines() if " w<=4 " in ln or " w<=7 " in ln]
    assert small and all("direct=-1.0" not in ln for ln in small), report
    h.close()


def test_direct_path_reports_unsupported(ctx):
    """While switched off, the direct path fails cleanly with CA_EUNSUPPORTED
    (no kernel is launched) and the tuner never times it."""
    import paper_2512_13133_amd as ca
    cs = small_window_set(64, 8, seed=3)
    h = ctx.clips(cs, image=True)
    with pytest.raises(ca.ClipAlignError) as e:
        ctx.align_pairs(h, [0], [1], "cosine", (19, 20), "direct")
    assert e.value.status == ca.CA_EUNSUPPORTED
    with pytest.raises(ca.ClipAlignError) as e:
        ctx.surface(h, [0], [1], path="direct")
    assert e.value.status == ca.CA_EUNSUPPORTED
    h.close()
