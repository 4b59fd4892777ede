"""Pins of the FP64 oracle against what the paper and mathematics fix.

None of these re-types the oracle's formula: each checks it against a closed
form (Fourier shift theorem, Parseval), a brute force over all shifts or all
covers, a worked example printed in the paper, or an independently written
textbook routine.
"""
import itertools
import json
import math
import os
from collections import deque
from fractions import Fraction

import numpy as np
import pytest
from scipy.fft import dctn

import clipgen
from oracle import cosine, cover, edge, loop, prune, raster, scp, serve, xcorr, xysep

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_clip(rng, N, k=4, lo=1):
    rects = []
    for _ in range(k):
        x0, x1 = sorted(rng.choice(N + 1, 2, replace=False))
        y0, y1 = sorted(rng.choice(N + 1, 2, replace=False))
        rects.append((x0, x1, y0, y1))
    return raster.rasterize(rects, N)


# ---------------------------------------------------------------- raster


def test_raster_half_open_and_clipping():
    a = raster.rasterize([(1, 3, 2, 4), (-5, 1, 7, 20)], 8)
    want = np.zeros((8, 8), bool)
    for y in range(8):
        for x in range(8):
            want[y, x] = (1 <= x < 3 and 2 <= y < 4) or (-5 <= x < 1 and 7 <= y < 20)
    assert (a == want).all()


def _flood_components(a):
    """Independent BFS labelling with 4-neighbourhood."""
    N = a.shape[0]
    lab = np.zeros(a.shape, int)
    nxt = 0
    for y in range(N):
        for x in range(N):
            if a[y, x] and not lab[y, x]:
                nxt += 1
                dq = deque([(y, x)])
                lab[y, x] = nxt
                while dq:
                    cy, cx = dq.popleft()
                    for ny, nx in ((cy + 1, cx), (cy - 1, cx), (cy, cx + 1), (cy, cx - 1)):
                        if 0 <= ny < N and 0 <= nx < N and a[ny, nx] and not lab[ny, nx]:
                            lab[ny, nx] = nxt
                            dq.append((ny, nx))
    return lab, nxt


def test_components_match_flood_fill():
    rng = np.random.default_rng(5)
    for _ in range(30):
        a = rng.random((12, 12)) < 0.45
        lab, boxes = raster.components(a)
        ref, P = _flood_components(a)
        assert boxes.shape[0] == P
        # same partition of pixels (labels may differ by permutation)
        pairs = set(zip(lab[a].tolist(), ref[a].tolist()))
        assert len(pairs) == P
        for p in range(1, P + 1):
            ys, xs = np.nonzero(lab == p)
            assert tuple(boxes[p - 1]) == (xs.min(), xs.max() + 1, ys.min(), ys.max() + 1)


# ---------------------------------------------------------------- cosine


def test_spectrum_equals_explicit_dft():
    rng = np.random.default_rng(1)
    N = 8
    a = rng.random((N, N)) < 0.5
    D = np.exp(-2j * np.pi * np.outer(np.arange(N), np.arange(N)) / N)
    F_ref = D @ a.astype(float) @ D.T  # sum_y sum_x a[y,x] e^{-2pi i (u y + v x)/N}
    assert np.allclose(cosine.spectrum(a), F_ref, atol=1e-12)


@pytest.mark.parametrize("N", [16, 32, 64])
def test_self_match_peaks_at_one_at_zero(N):
    rng = np.random.default_rng(N)
    for _ in range(5):
        a = rand_clip(rng, N)
        if a.sum() == 0:
            continue
        W = cosine.whiten(cosine.spectrum(a))
        res = cosine.align(a, a, W, W, N // 4, 19, 20)
        assert res["s"] == (0, 0)
        assert abs(res["r1"] - 1.0) < 1e-12
        assert res["c"] == a.sum() and res["score"] == 1.0 and res["bit"]


@pytest.mark.parametrize("N,w", [(16, 3), (32, 8), (64, 8)])
def test_cyclic_shift_recovered_exactly(N, w):
    """Fourier shift theorem (Eqs. 3-5): g = f shifted by t gives a unit delta at t."""
    rng = np.random.default_rng(100 + N)
    for _ in range(6):
        f = rand_clip(rng, N)
        if f.sum() == 0:
            continue
        t = tuple(int(v) for v in rng.integers(-w, w + 1, size=2))
        g = np.roll(f, shift=t, axis=(0, 1))  # g(x) = f(x - t)
        Wf, Wg = (cosine.whiten(cosine.spectrum(x)) for x in (f, g))
        r, K = cosine.surface(Wg, Wf)
        assert abs(r[t[0] % N, t[1] % N] - 1.0) < 1e-12
        # off the peak only the whitened-out bins remain: |r| <= (N^2 - K)/K < 1
        off = r.copy()
        off[t[0] % N, t[1] % N] = 0
        assert np.abs(off).max() <= (N * N - K) / K + 1e-12
        res = cosine.align(g, f, Wg, Wf, w, 19, 20)
        assert res["s"] == t and res["c"] == f.sum()


@pytest.mark.parametrize("N", [8, 16])
def test_surface_equals_spatial_correlation_of_whitened_images(N):
    """r(s) = (N^2/K) sum_x w_rep(x) w_mem(x+s), w = inverse DFT of the whitened spectrum."""
    rng = np.random.default_rng(7 + N)
    for _ in range(4):
        a, b = rand_clip(rng, N), rand_clip(rng, N)
        if a.sum() == 0 or b.sum() == 0:
            continue
        Wa, Wb = (cosine.whiten(cosine.spectrum(x)) for x in (a, b))
        r, K = cosine.surface(Wa, Wb)  # member a, rep b
        wa = np.fft.ifft2(Wa)
        wb = np.fft.ifft2(Wb)
        for dy in range(N):
            for dx in range(N):
                acc = 0j
                for y in range(N):
                    for x in range(N):
                        acc += np.conj(wb[y, x]) * wa[(y + dy) % N, (x + dx) % N]
                assert abs(acc.real * N * N / K - r[dy, dx]) < 1e-12
        # and the term-by-term sum of Eq. 5 at a few shifts
        sh = [(0, 0), (1, -2), (-3, 3)]
        assert np.allclose(cosine.surface_at(Wa, Wb, sh), [r[dy % N, dx % N] for dy, dx in sh], atol=1e-12)


def test_whitened_image_closed_forms():
    """A single set pixel has |F| = 1 at every bin, so W = F and the image is
    N at that pixel and 0 elsewhere; energy equals the non-zero bin count
    (Parseval); and the image equals the explicit inverse DFT sum."""
    for N in (8, 16, 64):
        a = np.zeros((N, N))
        a[3, N - 2] = 1
        img = cosine.whitened_image(cosine.whiten(cosine.spectrum(a)))
        ref = np.zeros((N, N))
        ref[3, N - 2] = N
        assert np.abs(img - ref).max() < 1e-12
    rng = np.random.default_rng(5)
    N = 8
    for _ in range(4):
        a = rand_clip(rng, N)
        W = cosine.whiten(cosine.spectrum(a))
        img = cosine.whitened_image(W)
        assert abs((img ** 2).sum() - np.count_nonzero(W)) < 1e-9
        for y, x in [(0, 0), (2, 5), (7, 1)]:
            acc = 0j
            for u in range(N):
                for v in range(N):
                    acc += W[u, v] * complex(math.cos(2 * math.pi * (u * y + v * x) / N),
                                             math.sin(2 * math.pi * (u * y + v * x) / N))
            assert abs(acc.imag) < 1e-9
            assert abs(acc.real / N - img[y, x]) < 1e-12


@pytest.mark.parametrize("N", [8, 16])
def test_image_correlation_is_the_surface(N):
    """sum_x img_rep(x) img_mem(x + s) = K r(s) at every shift, against an
    explicit quadruple loop (no array rolls)."""
    rng = np.random.default_rng(17 + N)
    for _ in range(3):
        a, b = rand_clip(rng, N), rand_clip(rng, N)
        if a.sum() == 0 or b.sum() == 0:
            continue
        Wa, Wb = (cosine.whiten(cosine.spectrum(x)) for x in (a, b))
        r, K = cosine.surface(Wa, Wb)  # member a, rep b
        ia, ib = cosine.whitened_image(Wa), cosine.whitened_image(Wb)
        shifts = [(dy, dx) for dy in range(-3, 4) for dx in range(-3, 4)]
        got = cosine.correlate_images(ia, ib, shifts)
        for (dy, dx), g in zip(shifts, got):
            acc = 0.0
            for y in range(N):
                for x in range(N):
                    acc += ib[y, x] * ia[(y + dy) % N, (x + dx) % N]
            assert abs(g - acc) < 1e-9
            assert abs(g / K - r[dy % N, dx % N]) < 1e-12


def test_surface_reverse_is_mirror():
    rng = np.random.default_rng(11)
    N = 32
    for _ in range(5):
        a, b = rand_clip(rng, N), rand_clip(rng, N)
        Wa, Wb = (cosine.whiten(cosine.spectrum(x)) for x in (a, b))
        r_ab, _ = cosine.surface(Wa, Wb)
        r_ba, _ = cosine.surface(Wb, Wa)
        idx = (-np.arange(N)) % N
        assert np.abs(r_ab - r_ba[np.ix_(idx, idx)]).max() < 1e-12


def test_window_residue_rule():
    assert list(cosine.window_axis(2, 8)) == [-2, -1, 0, 1, 2]
    assert list(cosine.window_axis(3, 7)) == [-3, -2, -1, 0, 1, 2, 3]
    assert list(cosine.window_axis(4, 8)) == [-4, -3, -2, -1, 0, 1, 2, 3]  # 9 > 8
    assert list(cosine.window_axis(32, 64)) == list(range(-32, 32))
    assert cosine.window(1, 8).shape == (9, 2)


def test_overlap_count_is_explicit_sum():
    rng = np.random.default_rng(3)
    N = 10
    a, b = rng.random((N, N)) < 0.4, rng.random((N, N)) < 0.6
    for dy in range(-4, 5):
        for dx in range(-4, 5):
            ref = sum(int(a[y, x] and b[(y + dy) % N, (x + dx) % N]) for y in range(N) for x in range(N))
            assert cosine.overlap(a, b, dy, dx) == ref


def test_argmax_and_tie_rule_brute_force():
    """Scan every window shift; pick max r, then within 1e-9: max c, min |s|_1, lex."""
    rng = np.random.default_rng(21)
    N, w = 16, 4
    # symmetric patterns create exact ties in r
    for trial in range(25):
        if trial % 3 == 0:
            h = rand_clip(rng, N // 2, k=2)
            a = np.zeros((N, N), bool)
            a[:N // 2, :N // 2] = h
            a[N // 2:, N // 2:] = h
            b = np.roll(a, (trial % 5, 1), axis=(0, 1))
        else:
            a, b = rand_clip(rng, N), rand_clip(rng, N)
        if a.sum() == 0 or b.sum() == 0:
            continue
        Wa, Wb = (cosine.whiten(cosine.spectrum(x)) for x in (a, b))
        res = cosine.align(a, b, Wa, Wb, w, 3, 4)
        shifts = [(dy, dx) for dy in range(-w, w + 1) for dx in range(-w, w + 1)]
        vals = cosine.surface_at(Wa, Wb, shifts)
        top = vals.max()
        cands = []
        for (dy, dx), v in zip(shifts, vals):
            if v >= top - 1e-9:
                c = sum(int(b[y, x] and a[(y + dy) % N, (x + dx) % N]) for y in range(N) for x in range(N))
                cands.append((-c, abs(dy) + abs(dx), dy, dx))
        best = min(cands)
        assert res["s"] == (best[2], best[3]) and res["c"] == -best[0]


def test_dct_parseval_reading_of_eq2():
    """Eq. 2 on orthonormal DCT-II coefficients equals the pixel cosine."""
    rng = np.random.default_rng(9)
    for _ in range(10):
        a, b = rand_clip(rng, 32), rand_clip(rng, 32)
        A, B = dctn(a.astype(float), norm="ortho"), dctn(b.astype(float), norm="ortho")
        dct_cos = (A * B).sum() / math.sqrt((A * A).sum() * (B * B).sum())
        c = int((a & b).sum())
        assert abs(dct_cos - cosine.score(c, int(a.sum()), int(b.sum()))) < 1e-12


def test_threshold_is_exact_rational():
    # c^2 / (n n) = 361/400 = 0.9025 = (19/20)^2 exactly: strict ">" fails
    assert cosine.bit(19, 20, 20, 19, 20) is False
    assert cosine.bit(20, 20, 21, 19, 20) is True  # 400/420 > 0.9025
    assert cosine.bit(0, 0, 5, 19, 20) is False
    assert cosine.score(19, 20, 20) == 0.95


# ---------------------------------------------------------------- edge


def test_minmax_worked_example_from_paper():
    g = json.load(open(os.path.join(GOLDEN, "minmax_worked_example.json")))
    s, E = edge.minmax_1d([g["d_min"], 7, 4, g["d_max"]], w=100)
    assert s == g["T_opt"] and E == g["E_min"]
    assert abs(g["d_min"] - s) == g["left_error"] and abs(g["d_max"] - s) == g["right_error"]


def test_minmax_1d_brute_force_with_tie_rule():
    rng = np.random.default_rng(4)
    for _ in range(400):
        ds = list(rng.integers(-20, 21, size=int(rng.integers(1, 7))))
        w = int(rng.integers(0, 25))
        best = min(range(-w, w + 1), key=lambda s: (max(abs(d - s) for d in ds), abs(s)))
        s, E = edge.minmax_1d(ds, w)
        assert s == best and E == max(abs(d - s) for d in ds)


def test_linf_separability_brute_force():
    """min over 2-D integer T of max_i |d_i - T|_inf equals max of the two 1-D solves."""
    rng = np.random.default_rng(8)
    for _ in range(100):
        dx = rng.integers(-9, 10, size=4)
        dy = rng.integers(-9, 10, size=4)
        w = 9
        brute = min(max(max(abs(int(a) - sx), abs(int(b) - sy)) for a, b in zip(dx, dy))
                    for sx in range(-w, w + 1) for sy in range(-w, w + 1))
        _, ex = edge.minmax_1d(dx, w)
        _, ey = edge.minmax_1d(dy, w)
        assert brute == max(ex, ey)


def test_translated_rectangles_align_exactly():
    N = 32
    for t in [(0, 0), (3, -2), (-5, 5)]:
        rep = raster.rasterize([(4, 12, 6, 10), (16, 20, 14, 28)], N)
        mem = raster.rasterize([(4 + t[1], 12 + t[1], 6 + t[0], 10 + t[0]),
                                (16 + t[1], 20 + t[1], 14 + t[0], 28 + t[0])], N)
        res = edge.align(mem, rep, 8, 0)
        assert res["s"] == t and res["E"] == 0 and res["bit"]


def _overlaps(mem_lab, rep_lab, p, q, dy, dx):
    N = rep_lab.shape[0]
    for y in range(N):
        for x in range(N):
            if rep_lab[y, x] == q and 0 <= y + dy < N and 0 <= x + dx < N and mem_lab[y + dy, x + dx] == p:
                return True
    return False


def test_edge_bit_brute_force_tiny():
    """Whenever the edge bit is set, an independent check confirms the rule at s."""
    rng = np.random.default_rng(12)
    N = 12
    seen = 0
    for _ in range(120):
        a = rand_clip(rng, N, k=int(rng.integers(1, 3)))
        b = np.roll(a, tuple(rng.integers(-2, 3, size=2)), axis=(0, 1))
        if rng.random() < 0.3:
            b = rand_clip(rng, N, k=2)
        if a.sum() == 0 or b.sum() == 0:
            continue
        res = edge.align(a, b, 3, 2)
        if not res["bit"]:
            continue
        seen += 1
        dy, dx = res["s"]
        la, P = _flood_components(a)
        lb, Q = _flood_components(b)
        fewer_a, fewer_b = P <= Q, Q <= P
        ds_x, ds_y = [], []
        for p in range(1, P + 1):
            hits = [q for q in range(1, Q + 1) if _overlaps(la, lb, p, q, dy, dx)]
            if fewer_a:
                assert len(hits) == 1
        for q in range(1, Q + 1):
            hits = [p for p in range(1, P + 1) if _overlaps(la, lb, p, q, dy, dx)]
            if fewer_b:
                assert len(hits) == 1
        # residual at s over matched bounding boxes
        for p in range(1, P + 1):
            for q in range(1, Q + 1):
                if _overlaps(la, lb, p, q, dy, dx):
                    ya, xa = np.nonzero(la == p)
                    yb, xb = np.nonzero(lb == q)
                    ds_x += [xa.min() - xb.min(), xa.max() - xb.max()]
                    ds_y += [ya.min() - yb.min(), ya.max() - yb.max()]
        E = max(max(abs(d - dx) for d in ds_x), max(abs(d - dy) for d in ds_y))
        assert E == res["E"] <= 2
    assert seen > 10


def _bars(spans, N=64, y0=10, y1=14):
    """A raster of full-height bars x[a, b) x y[y0, y1): one polygon per span."""
    return raster.rasterize([(a, b, y0, y1) for a, b in spans], N)


def test_edge_correspondence_is_taken_at_T0():
    """Hand-worked (Sec. 2.2.2 with the T0 reading).  The member is the rep
    moved 8 px right: rep bars x[2,8), x[10,16); member bars x[10,16), x[18,24).
    Global boxes give d = (10-2, 24-16) = (8, 8), so T0 = (0, 8); there each
    rep bar lands on exactly one member bar, the matched edges all move by 8,
    so s = (0, 8) and E = 0.  Taken at s = 0 instead, rep bar x[2,8) meets no
    member bar and the pair would have no correspondence."""
    rep, mem = _bars([(2, 8), (10, 16)]), _bars([(10, 16), (18, 24)])
    assert edge.align(mem, rep, 16, 0) == dict(s=(0, 8), E=0, bit=True, ok=True)
    # the mirror direction: rep and member swap roles, the shift flips
    assert edge.align(rep, mem, 16, 0) == dict(s=(0, -8), E=0, bit=True, ok=True)


def test_edge_unmatched_polygon_moves_T0_but_not_E():
    """Hand-worked.  Rep bars x[10,20), x[30,40); the member has the same two
    bars plus an extra bar x[50,52) (3 > 2 polygons, so only the rep side must
    match).  Global boxes: d = (10-10, 52-40) = (0, 12), T0 = (0, 6): rep bar
    x[10,20) lands on x[16,26) (meets x[10,20) only), x[30,40) on x[36,46)
    (meets x[30,40) only).  The matched pairs have all displacements 0, so
    s = (0, 0) and E = 0: the extra bar moved T0 but enters no edge pair."""
    rep, mem = _bars([(10, 20), (30, 40)]), _bars([(10, 20), (30, 40), (50, 52)])
    assert edge.align(mem, rep, 16, 0) == dict(s=(0, 0), E=0, bit=True, ok=True)


def test_edge_recheck_change_clears_the_bit():
    """Hand-worked.  Rep bars q1 = x[20,30), q2 = x[40,53); member bars
    p0 = x[1,2), p1 = x[20,30), p2 = x[40,50), p3 = x[51,53).
    T0: d = (1-20, 53-53) = (-19, 0), half toward zero -> -9.  At T0 q1 lands
    on x[11,21) (meets p1 only), q2 on x[31,44) (meets p2 only): matching
    {(p1,q1), (p2,q2)}.  Edge displacements 0, 0 and 0, 50-53 = -3 give
    s_x = -1 (-3/2 toward zero), E = max(0+1, -1+3) = 2.  At s = (0, -1) q2
    lands on x[39,52) and meets p2 and p3, so the matching changed: no bit,
    although E = 2 <= T_edge = 2."""
    rep = _bars([(20, 30), (40, 53)])
    mem = _bars([(1, 2), (20, 30), (40, 50), (51, 53)])
    assert edge.align(mem, rep, 16, 2) == dict(s=(0, -1), E=2, bit=False, ok=False)
    # with p3 one pixel further right (x[52,54)) T0 is still -9 (d = (-19, 1)),
    # the matching and the solve are the same, q2 at x[39,52) now misses p3,
    # and the bit is set
    mem_ok = _bars([(1, 2), (20, 30), (40, 50), (52, 54)])
    assert edge.align(mem_ok, rep, 16, 2) == dict(s=(0, -1), E=2, bit=True, ok=True)


# ---------------------------------------------------------------- XY separation (cosine track)


def test_xysep_picks_the_narrowest_interval_per_axis():
    """Hand-worked (Sec. 3.2.1(2)).  Rep boxes A = x[10,20) y[10,20) and
    B = x[40,60) y[40,50); member boxes A' = x[14,23) y[11,22) and
    B' = x[42,62) y[43,53).  T0 from the global boxes (d_x = 4, 2 -> 3;
    d_y = 1, 3 -> 2) puts A' on A and B' on B only.  Intervals: A' x [3, 4]
    (Q 1), y [1, 2] (Q 1); B' x [2, 2] (Q 0), y [3, 3] (Q 0).  B' wins both
    axes: s = (3, 2).  The edge track's Min-Max over all edges gives (2, 3)
    instead, and so does T0."""
    N = 64
    rep = raster.rasterize([(10, 20, 10, 20), (40, 60, 40, 50)], N)
    mem = raster.rasterize([(14, 23, 11, 22), (42, 62, 43, 53)], N)
    (s, matched) = xysep.shift(mem, rep, 8)
    assert s == (3, 2) and matched
    assert edge.align(mem, rep, 8, 10)["s"] == (2, 3)
    res = xysep.align(mem, rep, 8, 19, 20)
    c = int(np.count_nonzero(rep & np.roll(mem, (-3, -2), axis=(0, 1))))
    assert res["s"] == (3, 2) and res["c"] == c
    assert res["score"] == c / math.sqrt(float(mem.sum()) * float(rep.sum()))


def test_xysep_ties_go_to_the_first_pair_and_windows_clamp():
    """Hand-worked.  Both pairs have x intervals of width 0 (A' d_x = 3,
    B' d_x = 2): the first pair in polygon order (A', the first in raster
    order) wins, s_x = 3; y: A' [1, 2] (Q 1) loses to B' [5, 5] (Q 0),
    s_y = 5.  With a half-window of 4 the y shift clamps to 4."""
    N = 64
    rep = raster.rasterize([(10, 20, 10, 20), (40, 60, 40, 50)], N)
    mem = raster.rasterize([(13, 23, 11, 22), (42, 62, 45, 55)], N)
    assert xysep.shift(mem, rep, 8) == ((5, 3), True)
    assert xysep.shift(mem, rep, 4) == ((4, 3), True)


def test_xysep_without_correspondence_uses_T0():
    """Hand-worked.  One rep bar x[10,30) against two member bars x[12,18)
    and x[22,28) (the rep is the fewer side and overlaps two member polygons
    at T0, so the exactly-one rule fails): the shift is T0 of the global
    boxes, d_x = 12-10, 28-30 = (2, -2) -> 0, d_y = 0 -> (0, 0)."""
    N = 64
    rep = _bars([(10, 30)])
    mem = _bars([(12, 18), (22, 28)])
    assert xysep.shift(mem, rep, 8) == ((0, 0), False)
    # an empty member: no shift, no count
    assert xysep.align(np.zeros_like(rep), rep, 8, 19, 20) == dict(s=(0, 0), c=0, score=0.0, bit=False,
                                                                     matched=False)


def test_xysep_recovers_translations_exactly():
    """Closed form: a clip translated by t inside its window (content away
    from the border, so every box moves by t) gives every interval [t, t], the
    shift t and c = n: a full match."""
    rng = np.random.default_rng(31)
    N, w = 64, 8
    for _ in range(40):
        rects = []
        for _ in range(int(rng.integers(1, 5))):
            x0, y0 = rng.integers(10, 40, 2)
            rects.append((int(x0), int(x0 + rng.integers(2, 12)), int(y0), int(y0 + rng.integers(2, 12))))
        rep = raster.rasterize(rects, N)
        ty, tx = (int(v) for v in rng.integers(-w, w + 1, 2))
        mem = np.roll(rep, (ty, tx), axis=(0, 1))
        res = xysep.align(mem, rep, w, 19, 20)
        assert res["s"] == (ty, tx) and res["c"] == int(rep.sum()) and res["bit"]


def test_xysep_names_residues_when_the_window_wraps():
    """C0 rule: with 2w + 1 > N every residue is named in [-N/2, N/2 - 1];
    a box pair displaced by +8 on a 16-grid with w = 8 gives the shift -8."""
    N = 16
    rep = raster.rasterize([(0, 4, 0, 4)], N)
    mem = raster.rasterize([(8, 12, 0, 4)], N)
    assert xysep.shift(mem, rep, 8) == ((0, -8), True)
    assert xysep.residue(8, 8, 16) == -8 and xysep.residue(7, 8, 16) == 7 and xysep.residue(8, 8, 64) == 8


# ---------------------------------------------------------------- pruning


def test_pruning_bounds_are_safe():
    rng = np.random.default_rng(13)
    N, w = 16, 3
    for _ in range(60):
        a, b = rand_clip(rng, N, k=3), rand_clip(rng, N, k=3)
        if a.sum() == 0 or b.sum() == 0:
            continue
        best = max(cosine.overlap(b, a, dy, dx) for dy in range(-w, w + 1) for dx in range(-w, w + 1))
        assert prune.signature_bound(a, b, w) >= best
        assert min(a.sum(), b.sum()) >= best
        Wa, Wb = (cosine.whiten(cosine.spectrum(x)) for x in (a, b))
        for p, q in [(19, 20), (3, 5), (1, 2)]:
            res = cosine.align(a, b, Wa, Wb, w, p, q)
            if res["bit"]:
                assert prune.area_pass(int(a.sum()), int(b.sum()), p, q)
                assert prune.signature_pass(a, b, w, p, q)


def test_bounds_over_many_pairs_equal_the_pairwise_bounds():
    """area_pairs lists exactly the pairs area_pass admits, and the batched B2
    bound equals the pairwise one, on random 16 x 16 clips."""
    rng = np.random.default_rng(23)
    N, w = 16, 3
    clips = [rand_clip(rng, N, k=int(rng.integers(1, 5))) for _ in range(30)]
    npix = np.array([int(c.sum()) for c in clips])
    for p, q in [(19, 20), (93, 100), (1, 2)]:
        r, m = prune.area_pairs(npix, p, q)
        got = set(zip(r.tolist(), m.tolist()))
        want = {(i, j) for i in range(30) for j in range(i + 1, 30) if prune.area_pass(npix[i], npix[j], p, q)}
        assert got == want
    a_idx, b_idx = rng.integers(0, 30, 80), rng.integers(0, 30, 80)
    rows = np.array([c.sum(axis=1) for c in clips]).astype(np.int64)
    cols = np.array([c.sum(axis=0) for c in clips]).astype(np.int64)
    many = prune.signature_bound_many(rows[a_idx], cols[a_idx], rows[b_idx], cols[b_idx], w)
    one = [prune.signature_bound(clips[i], clips[j], w) for i, j in zip(a_idx, b_idx)]
    assert many.tolist() == one
    ok = prune.signature_pass_many(rows[a_idx], cols[a_idx], npix[a_idx], rows[b_idx], cols[b_idx], npix[b_idx],
                                   w, 19, 20)
    assert ok.tolist() == [prune.signature_pass(clips[i], clips[j], w, 19, 20) for i, j in zip(a_idx, b_idx)]


def test_edge_box_bound_is_safe():
    rng = np.random.default_rng(14)
    N = 16
    for _ in range(80):
        a = rand_clip(rng, N, k=2)
        b = np.roll(a, tuple(rng.integers(-2, 3, size=2)), axis=(0, 1)) if rng.random() < 0.5 else rand_clip(rng, N, k=2)
        if a.sum() == 0 or b.sum() == 0:
            continue
        for t in (0, 1, 2):
            res = edge.align(a, b, 4, t)
            if res["bit"]:
                assert prune.edge_pair_pass(raster.components(a)[1], raster.components(b)[1], t)


# ---------------------------------------------------------------- set cover


def _chvatal(n, covers):
    """Textbook greedy set cover: sets are {j} + out(j); pick the set covering the
    most uncovered elements, lowest index on ties."""
    sets = [set([j]) | set(np.flatnonzero(covers[j]).tolist()) for j in range(n)]
    U, chosen = set(range(n)), []
    while U:
        j = max((j for j in range(n) if j in U), key=lambda j: (len(sets[j] & U), -j))
        chosen.append(j)
        U -= sets[j]
    return chosen


def _random_cover(rng, n, p):
    cov = rng.random((n, n)) < p
    np.fill_diagonal(cov, True)
    return cov


def test_lazy_equals_eager():
    rng = np.random.default_rng(15)
    for _ in range(40):
        n = int(rng.integers(1, 40))
        cov = _random_cover(rng, n, rng.uniform(0.02, 0.4))
        if rng.random() < 0.5:
            cov = cov | cov.T
        pool = np.sort(rng.choice(n, size=int(rng.integers(1, n + 1)), replace=False))
        assert scp.lazy(pool, cov) == scp.eager(pool, cov)


def test_surprisal_reduces_to_chvatal_on_regular_graphs():
    """Equal in-degrees make every S_i equal, so Score_j ranks like |covered|."""
    rng = np.random.default_rng(16)
    for n, d in [(12, 2), (20, 4), (31, 6)]:
        for _ in range(5):
            perm = rng.permutation(n)
            cov = np.zeros((n, n), bool)
            for k in range(1, d + 1):  # circulant: i covers i+k -> every in-degree is d
                cov[perm, perm[(np.arange(n) + k) % n]] = True
            np.fill_diagonal(cov, True)
            reps, _ = scp.lazy(np.arange(n), cov)
            assert reps == _chvatal(n, cov & ~np.eye(n, dtype=bool))


def test_cover_result_is_a_partition():
    rng = np.random.default_rng(17)
    for _ in range(20):
        n = 30
        cov = _random_cover(rng, n, 0.1)
        reps, assign = scp.lazy(np.arange(n), cov)
        assert sorted(assign) == list(range(n))
        for i, r in assign.items():
            assert cov[r, i] and assign[r] == r
        assert set(reps) == set(assign.values())


def test_surprisal_prefers_rare_nodes():
    """A hub covering 3 common nodes loses to one covering 2 rare nodes."""
    n = 8
    cov = np.eye(n, dtype=bool)
    cov[0, [1, 2, 3]] = True  # hub 0
    for j in (4, 5, 6):  # 1,2,3 are each covered by many
        cov[j, [1, 2, 3]] = True
    cov[7, [4, 5]] = True  # 7 covers nodes that only 0.. nobody else covers
    reps, _ = scp.eager(np.arange(n), cov)
    # Score_7 = 1 + 1/2 + 1/2 (4,5 each covered only by 7) beats Score_0 = 1 + 3 * 1/5
    assert reps[0] == 7


# ---------------------------------------------------------------- loop


def test_loop_single_iteration_is_set_cover():
    rng = np.random.default_rng(18)
    n = 25
    cov = _random_cover(rng, n, 0.15)
    rep_of, reps, _ = loop.run(n, lambda tau: cov, [None])
    r2, assign = scp.lazy(np.arange(n), cov)
    assert reps == r2 and all(rep_of[i] == assign[i] for i in range(n))


def test_loop_converges_and_members_pass_strict():
    rng = np.random.default_rng(19)
    n = 40
    scores = rng.random((n, n))
    scores = np.maximum(scores, scores.T)
    np.fill_diagonal(scores, 9)

    def bits_at(tau):
        return scores >= tau

    rep_of, reps, log = loop.run(n, bits_at, [0.6, 0.75, 0.9])
    strict = bits_at(0.9)
    assert (rep_of >= 0).all()
    for i in range(n):
        assert strict[rep_of[i], i] and rep_of[rep_of[i]] == rep_of[i]
    assert len(set(rep_of.tolist())) == len(reps)


def test_loop_reattaches_to_first_selected_representative():
    """Hand-worked (Sec. 3.1 stages 3-4 with the re-attachment reading).
    Ten nodes, K = 2.  Strict covers: 0 -> {4, 5, 6}, 2 -> {3, 7, 9},
    1 -> {3, 8}; the relaxed graph adds 0 -> 3.
    Iteration 1 (relaxed): in-degrees give f_3 = 4, f_4..f_9 = 2, f_0..f_2 = 1,
    so Score_0 = 1 + 1/4 + 3/2 = 2.75 > Score_2 = 2.25 > Score_1 = 1.75: node 0
    is selected and takes 3, 4, 5, 6; then Score_2 = 1 + 1/2 + 1/2 = 2 beats
    Score_1 = 1.5.  Selection order [0, 2, 1].  Refinement: 0 does not cover 3
    strictly, so 3 is the only orphan.
    Iteration 2 (strict): 3 re-attaches to the first representative in
    selection order that covers it strictly, 2 (not 1, the lower id and the
    last one selected); skipping re-attachment would make 3 its own
    representative."""
    n = 10
    strict = np.eye(n, dtype=bool)
    for j, ks in {0: [4, 5, 6], 2: [3, 7, 9], 1: [3, 8]}.items():
        strict[j, ks] = True
    relaxed = strict.copy()
    relaxed[0, 3] = True
    rep_of, reps, log = loop.run(n, lambda tau: relaxed if tau == "relaxed" else strict, ["relaxed", "strict"])
    assert reps == [0, 2, 1]
    assert rep_of.tolist() == [0, 1, 2, 2, 0, 0, 0, 2, 1, 2]
    assert [(g["pool"], g["selected"], g["orphans"]) for g in log] == [(10, 3, 1), (0, 0, 0)]


def test_schedules():
    assert loop.cosine_schedule(19, 20, 3) == [(93, 100), (47, 50), (19, 20)]
    assert loop.cosine_schedule(19, 20, 1) == [(19, 20)]
    assert loop.edge_schedule(2, 3) == [4, 3, 2]
    # other relaxations: 0.95 - 0.03 (4 - t)/3 = 0.92, 0.93, 0.94, 0.95; 2 px a step
    assert loop.cosine_schedule(19, 20, 4, Fraction(3, 100)) == [(23, 25), (93, 100), (47, 50), (19, 20)]
    assert loop.edge_schedule(2, 3, 2) == [6, 4, 2]
    assert loop.cosine_schedule(19, 20, 3, 0) == [(19, 20)] * 3


def test_loop_without_relaxation_is_one_set_cover():
    """With no relaxation every iteration uses the strict threshold: the
    first set cover places every node and the later iterations find an empty
    pool, so K iterations give the K = 1 result."""
    rng = np.random.default_rng(20)
    n = 30
    cov = _random_cover(rng, n, 0.2)
    one = loop.run(n, lambda tau: cov, [None])
    three = loop.run(n, lambda tau: cov, [None, None, None])
    assert one[1] == three[1] and (one[0] == three[0]).all()
    assert [g["pool"] for g in three[2]] == [n, 0, 0]


# ---------------------------------------------------------------- drivers


def test_small_workload_symmetry_and_cover():
    cs = clipgen.small(n_clips=40)
    rep, mem = clipgen.all_pairs(cs.n)
    res = cover.align_pairs_cosine(cs, rep, mem, 19, 20)
    # equal windows: the relation and the shifts are mirror-symmetric
    assert ((res["bits"] & 1) == (res["bits"] >> 1)).all()
    assert (res["shift"][:, 0] == -res["shift"][:, 1]).all()
    assert (res["c"][:, 0] == res["c"][:, 1]).all()
    er = cover.align_pairs_edge(cs, rep, mem, 2)
    assert ((er["bits"] & 1) == (er["bits"] >> 1)).all()
    cl = cover.cluster_cosine(cs, 19, 20, K=1, rep=rep, mem=mem, res=res)
    assert 1 <= cl["n_clusters"] <= cs.n


# ------------------------------------------------------------------ exact objective (NEXT f1)


@pytest.mark.parametrize("N,w", [(32, 5), (64, 16)])
def test_xcorr_counts_equal_fft_correlation(N, w):
    """c(s) from the definition equals the circular cross-correlation of the
    two rasters computed through numpy's FFT (rounded to integers) at every
    shift of the window."""
    rng = np.random.default_rng(N + w)
    for _ in range(3):
        a_m = rand_clip(rng, N, k=5)
        a_r = rand_clip(rng, N, k=5)
        shifts, counts = xcorr.overlap_surface(a_m, a_r, w)
        corr = np.fft.ifft2(np.conj(np.fft.fft2(a_r.astype(float))) * np.fft.fft2(a_m.astype(float))).real
        ref = np.rint(corr[shifts[:, 0] % N, shifts[:, 1] % N]).astype(np.int64)
        assert (counts == ref).all()


def test_xcorr_recovers_cyclic_shift_exactly():
    """A member that is the representative moved by s0 (inside the window)
    aligns at s0 with c = n: no other shift can reach all n pixels of a dense
    random pattern."""
    rng = np.random.default_rng(9)
    N, w = 64, 12
    for s0 in [(0, 0), (3, -7), (-12, 12), (5, 0)]:
        a_r = rng.random((N, N)) < 0.4
        a_m = np.roll(a_r, s0, axis=(0, 1))
        res = xcorr.align(a_m, a_r, w, 19, 20)
        assert res["s"] == s0 and res["c"] == int(a_r.sum()) and res["bit"]


def test_xcorr_tie_rule_on_constructed_ties():
    """One representative pixel against two member pixels: c = 1 at exactly
    two shifts, and the rule picks the smaller |dy|+|dx|, then the smaller
    (dy, dx)."""
    N, w = 32, 6
    a_r = np.zeros((N, N), bool)
    a_r[10, 10] = True
    for pix, want in [(((10, 13), (10, 7)), (0, -3)),   # equal |s|: smaller dx
                      (((13, 10), (10, 7)), (0, -3)),   # equal |s|: smaller dy first
                      (((12, 10), (10, 7)), (2, 0))]:   # smaller |dy| + |dx|
        a_m = np.zeros((N, N), bool)
        for y, x in pix:
            a_m[y, x] = True
        res = xcorr.align(a_m, a_r, w, 1, 2)
        assert res["s"] == want and res["c"] == 1


def test_xcorr_mirror_and_dominance():
    """c of (member, rep) at s equals c of (rep, member) at -s; the chosen
    overlap is never below the one phase correlation picks (same window)."""
    rng = np.random.default_rng(4)
    N, w = 32, 6
    for _ in range(4):
        a = rand_clip(rng, N, k=6)
        b = rand_clip(rng, N, k=6)
        s1, c1 = xcorr.overlap_surface(a, b, w)
        s2, c2 = xcorr.overlap_surface(b, a, w)
        m2 = {(int(dy), int(dx)): int(c) for (dy, dx), c in zip(s2, c2)}
        assert all(m2[(-int(dy), -int(dx))] == int(c) for (dy, dx), c in zip(s1, c1))
        if a.any() and b.any():
            pcm = cosine.align(a, b, cosine.whiten(cosine.spectrum(a)), cosine.whiten(cosine.spectrum(b)), w, 1, 2)
            assert xcorr.align(a, b, w, 1, 2)["c"] >= pcm["c"]



# ---------------------------------------------------------------- serving rule


def test_serve_best_match_rule_on_a_table():
    """The rule on hand-made pair results: request 0 is covered by library
    clips 5 (0.96) and 2 (0.97) -> 2; request 1 by 7 and 3 with equal scores
    -> 3 (lowest id), while library clip 1 scores higher without covering;
    request 2 is covered by nobody -> -1."""
    req = [0, 0, 1, 1, 1, 2, 0]
    lib = [5, 2, 7, 3, 1, 4, 9]
    bits = [True, True, True, True, False, False, False]
    score = [0.96, 0.97, 0.99, 0.99, 1.0, 0.5, 0.999]
    shift = [(1, 1), (2, -1), (0, 3), (-3, 0), (5, 5), (0, 0), (7, 7)]
    best, sc, sh, matched = serve.best_match(3, req, lib, bits, score, np.array(shift))
    assert best.tolist() == [2, 3, -1]
    assert sc.tolist() == [0.97, 0.99, 0.0]
    assert sh.tolist() == [[2, -1], [-3, 0], [0, 0]]
    assert matched.tolist() == [1, 1, 0]


def test_serve_match_on_translated_copies():
    """End to end on 32 x 32 clips: the request clip R is a 6 x 6 square;
    library clip 1 is R moved by (+1, +1) and clip 2 is R moved by (-2, 0),
    both cover R with score exactly 1, so the lower id 1 wins and R's shift
    relative to it is (-1, -1); library clip 0 (a 2 x 2 square) covers
    nothing.  A second request clip (a 1 x 1 dot) matches no library clip."""
    def cs(rect_lists):
        ptr = np.cumsum([0] + [len(r) for r in rect_lists]).astype(np.int64)
        rects = np.array([r for rl in rect_lists for r in rl], np.int32).reshape(-1, 4)
        n = len(rect_lists)
        return clipgen.ClipSet(ptr, rects, np.full(n, 32, np.int16), np.full(n, 4, np.int16),
                               np.zeros(n, np.int32), np.zeros((n, 2), np.int16))
    library = cs([[(0, 2, 0, 2)], [(11, 17, 11, 17)], [(10, 16, 8, 14)]])
    request = cs([[(10, 16, 10, 16)], [(25, 26, 25, 26)]])
    best, sc, sh, matched = serve.serve_match(library, request, 19, 20)
    assert best.tolist() == [1, -1] and matched.tolist() == [1, 0]
    assert sc.tolist() == [1.0, 0.0] and sh.tolist() == [[-1, -1], [0, 0]]



# ---------------------------------------------------------------- cover relation and centers


def test_cover_csr_lists_each_set_direction_once_sorted():
    """Hand-made results of three pairs on five clips: (0,3) both directions,
    (4,1) only 4 covers 1, (2,0) only 0 covers 2."""
    rep = [0, 4, 2]
    mem = [3, 1, 0]
    bits = [3, 1, 2]
    shift = np.array([[[1, 2], [-1, -2]], [[0, 5], [0, -5]], [[7, 7], [3, -3]]])
    value = [[10, 10], [8, 9], [1, 4]]
    score = [[0.9, 0.9], [0.8, 0.7], [0.1, 0.4]]
    out = cover.cover_csr(5, rep, mem, bits, shift, value, score)
    assert out["row_ptr"].tolist() == [0, 2, 2, 2, 3, 4]
    assert out["col"].tolist() == [2, 3, 0, 1]
    assert out["shift"].tolist() == [[3, -3], [1, 2], [-1, -2], [0, 5]]
    assert out["value"].tolist() == [4, 10, 10, 8]
    assert out["score"].tolist() == [0.4, 0.9, 0.9, 0.8]


def test_oracle_clusters_pass_center_verification_and_planted_errors_fail():
    """Every assignment the closed loop produces satisfies the strict
    constraint at its centers (K = 1 and 3, both tracks); moving a member to a
    clip that does not cover it, shifting it off its center, or naming a
    non-representative as representative is reported."""
    cs = clipgen.small(n_clips=40)
    rep, mem = clipgen.all_pairs(cs.n)
    res = cover.align_pairs_cosine(cs, rep, mem, 19, 20)
    er = cover.align_pairs_edge(cs, rep, mem, 2)
    for K in (1, 3):
        cl = cover.cluster_cosine(cs, 19, 20, K=K, rep=rep, mem=mem, res=res)
        assert cover.verify_centers(cs, cl["rep_of"], cl["shift"], "cosine", (19, 20)) == []
        ce = cover.cluster_edge(cs, 2, K=K, rep=rep, mem=mem, res=er)
        assert cover.verify_centers(cs, ce["rep_of"], ce["shift"], "edge", 2) == []
    cl = cover.cluster_cosine(cs, 19, 20, K=1, rep=rep, mem=mem, res=res)
    rep_of, sh = cl["rep_of"].copy(), cl["shift"].copy()
    members = [i for i in range(cs.n) if rep_of[i] != i]
    assert members
    i = members[0]
    r = int(rep_of[i])
    # a representative that does not cover i at any shift of its window
    others = [j for j in range(cs.n) if rep_of[j] == j and j != r]
    a_i = raster.clip_raster(cs, i)
    far = next(j for j in others
               if not any(cosine.bit(cosine.overlap(raster.clip_raster(cs, j), a_i, dy, dx), int(a_i.sum()),
                                     int(raster.clip_raster(cs, j).sum()), 19, 20)
                          for dy, dx in cosine.window(int(cs.marker_w[i]), 64)))
    moved = rep_of.copy()
    moved[i] = far
    assert cover.verify_centers(cs, moved, sh, "cosine", (19, 20)) == [i]
    off = sh.copy()
    off[i] = (9, 9)  # outside the 17 x 17 window
    assert cover.verify_centers(cs, rep_of, off, "cosine", (19, 20)) == [i]
    chain = rep_of.copy()
    chain[r] = i  # r no longer represents itself: r and its members fail
    bad = cover.verify_centers(cs, chain, sh, "cosine", (19, 20))
    assert r in bad and i in bad
