"""Pins of the full boundary-edge oracle (`oracle/contour.py`, paper
Sec. 2.2.2 edge movement constraint over all corresponding edges; Sec. 3.1
stage 1 topological hashing).

Each check is independent of the tracing code: side counts and corner classes
from numpy differences, hole counts from an 8-connected labelling of the
complement (digital topology pairs 4-connected sets with 8-connected
complements), hand-worked shapes (fixture `golden/contour_worked_example.json`),
translation invariance, the reduction to the bounding-box track when every
polygon is a rectangle, a published FNV-1a test vector, and the pre-filter
never dropping a pair that meets the constraint.
"""
import json
import os

import numpy as np
import pytest
from scipy import ndimage

import clipgen
from oracle import contour, cover, edge, raster

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
EIGHT = np.ones((3, 3), dtype=bool)


def masks_of(a):
    lab, boxes = raster.components(a)
    return [lab == p for p in range(1, boxes.shape[0] + 1)]


def random_raster(rng, N, k):
    rects = []
    for _ in range(k):
        x0 = int(rng.integers(0, N - 1))
        y0 = int(rng.integers(0, N - 1))
        rects.append((x0, x0 + int(rng.integers(1, N // 2)), y0, y0 + int(rng.integers(1, N // 2))))
    return raster.rasterize(rects, N)


def boundary_side_count(m):
    """Unit sides between the mask and its complement (outside = 0)."""
    p = np.pad(m, 1).astype(np.int8)
    return int(np.abs(np.diff(p, axis=0)).sum() + np.abs(np.diff(p, axis=1)).sum())


def corner_vertex_count(m):
    """Contour vertices from 2x2 corner windows: one per corner with 1 or 3
    set pixels, two per diagonal pair."""
    p = np.pad(m, 1).astype(np.int8)
    a, b, c, d = p[:-1, :-1], p[:-1, 1:], p[1:, :-1], p[1:, 1:]
    s = a + b + c + d
    diag = ((a & d & (1 - b) & (1 - c)) | (b & c & (1 - a) & (1 - d))).astype(bool)
    return int(((s == 1) | (s == 3)).sum() + 2 * diag.sum())


def hole_count(m):
    """8-connected components of the complement that do not reach the border."""
    comp = ~np.pad(m, 1)
    lab, n = ndimage.label(comp, structure=EIGHT)
    return n - 1  # the padded border is one component


def edge_lengths(con):
    n = len(con)
    out = []
    for k in range(n):
        _, x, y = con[k]
        _, x2, y2 = con[(k + 1) % n]
        out.append(abs(x2 - x) + abs(y2 - y))
    return out


# ------------------------------------------------------------ hand-worked


def test_single_pixel_and_rectangle():
    a = raster.rasterize([(2, 3, 5, 6)], 8)
    cons = contour.contours(a)
    assert cons == [[(0, 2, 5), (1, 3, 5), (2, 3, 6), (3, 2, 6)]]
    assert contour.turning(cons[0]) == 4
    r = raster.rasterize([(1, 6, 2, 4)], 8)   # x in [1, 6), y in [2, 4)
    poly = contour.polygon(r)
    # top (east) at y0, right (south) at x1, bottom (west) at y1, left (north) at x0
    assert poly == [[(0, 2), (1, 6), (2, 4), (3, 1)]]


def test_worked_examples_fixture():
    """Hand-worked L and U shapes: contours, canonical order, residuals (the
    U with a deeper notch has the bounding boxes of the original, so the box
    track sees E = 0 while the full-edge track sees E = 1)."""
    with open(os.path.join(GOLDEN, "contour_worked_example.json")) as f:
        ex = json.load(f)
    for case in ex["cases"]:
        N = case["N"]
        a_rep = raster.rasterize(case["rep_rects"], N)
        a_mem = raster.rasterize(case["mem_rects"], N)
        assert [list(map(list, c)) for c in contour.polygon(a_rep)] == case["rep_polygon"], case["name"]
        assert [list(map(list, c)) for c in contour.polygon(a_mem)] == case["mem_polygon"], case["name"]
        got = contour.align(a_mem, a_rep, case["w"], case["t_edge"])
        assert list(got["s"]) == case["shift"] and got["E"] == case["E"] and got["bit"] == case["bit"], case["name"]
        box = edge.align(a_mem, a_rep, case["w"], case["t_edge"])
        assert box["E"] == case["E_box"], case["name"]


def test_ring_has_one_hole_traversed_left():
    a = raster.rasterize([(1, 6, 1, 2), (1, 6, 5, 6), (1, 2, 1, 6), (5, 6, 1, 6)], 8)  # 5 x 5 ring
    poly = contour.polygon(a)
    assert len(poly) == 2
    cons = contour.contours(a)
    assert sorted(contour.turning(c) for c in cons) == [-4, 4]
    # the hole [2, 5) x [2, 5): its least rotation starts with its bottom side
    # run east (y = 5), then north at x = 5, west at y = 2, south at x = 2
    assert poly[1] == [(0, 5), (3, 5), (2, 2), (1, 2)]


def test_diagonal_touch_inside_one_polygon_turns_right():
    """A polygon whose own pixels meet diagonally at one corner: the enclosed
    background pixel reaches the outside diagonally, so it is no hole (one
    contour), and that corner is visited twice."""
    a = np.array([[1, 1, 1, 0],
                  [1, 1, 0, 0],
                  [1, 0, 1, 1],
                  [1, 1, 1, 1]], dtype=bool)
    assert raster.components(a)[1].shape[0] == 1
    cons = contour.contours(a)
    assert len(cons) == 1 and contour.turning(cons[0]) == 4
    starts = [(x, y) for _, x, y in cons[0]]
    assert starts.count((2, 2)) == 2
    assert hole_count(a) == 0


def test_fnv1a_published_vector():
    assert contour.fnv1a64(b"") == 0xCBF29CE484222325
    assert contour.fnv1a64(b"a") == 0xAF63DC4C8601EC8C


# ------------------------------------------------------------ invariants


@pytest.mark.parametrize("seed", range(6))
def test_counts_match_independent_definitions(seed):
    rng = np.random.default_rng(100 + seed)
    for _ in range(10):
        a = random_raster(rng, 24, int(rng.integers(2, 9)))
        for m in masks_of(a):
            cons = contour.contours(m)
            assert sum(sum(edge_lengths(c)) for c in cons) == boundary_side_count(m)
            assert sum(len(c) for c in cons) == corner_vertex_count(m)
            turns = sorted(contour.turning(c) for c in cons)
            assert turns.count(4) == 1 and turns.count(-4) == len(turns) - 1
            assert len(cons) - 1 == hole_count(m)
            # consecutive edges alternate horizontal and vertical
            for c in cons:
                assert all((c[k][0] - c[k - 1][0]) % 2 == 1 for k in range(len(c)))


def test_canonical_order_is_translation_invariant():
    rng = np.random.default_rng(7)
    for _ in range(20):
        a = random_raster(rng, 20, 5)
        big = np.zeros((32, 32), bool)
        ty, tx = int(rng.integers(0, 12)), int(rng.integers(0, 12))
        big[ty:ty + 20, tx:tx + 20] = a
        small = np.zeros((32, 32), bool)
        small[:20, :20] = a
        for m0, m1 in zip(masks_of(small), masks_of(big)):
            p0, p1 = contour.polygon(m0), contour.polygon(m1)
            assert contour.descriptor(p0) == contour.descriptor(p1)
            assert contour.poly_hash(p0) == contour.poly_hash(p1)
            for c0, c1 in zip(p0, p1):
                for (d, u0), (_, u1) in zip(c0, c1):
                    assert u1 - u0 == (tx if d in (contour.S_, contour.N_) else ty)


def test_pure_translation_aligns_exactly():
    rng = np.random.default_rng(11)
    for _ in range(20):
        a = random_raster(rng, 20, 4)
        ty, tx = int(rng.integers(-4, 5)), int(rng.integers(-4, 5))
        rep = np.zeros((32, 32), bool)
        mem = np.zeros((32, 32), bool)
        rep[6:26, 6:26] = a
        mem[6 + ty:26 + ty, 6 + tx:26 + tx] = a
        got = contour.align(mem, rep, 5, 0)
        assert got["E"] == 0 and got["bit"] and got["s"] == (ty, tx)


def separated_rectangles(rng, N, k):
    """Rectangles kept two pixels apart, so each is its own polygon."""
    occ = np.zeros((N, N), bool)
    rects = []
    for _ in range(50):
        if len(rects) == k:
            break
        w, h = int(rng.integers(2, 10)), int(rng.integers(2, 10))
        x0, y0 = int(rng.integers(0, N - w)), int(rng.integers(0, N - h))
        if occ[max(0, y0 - 2):y0 + h + 2, max(0, x0 - 2):x0 + w + 2].any():
            continue
        occ[y0:y0 + h, x0:x0 + w] = True
        rects.append((x0, x0 + w, y0, y0 + h))
    return rects


def test_rectangles_reduce_to_the_box_track():
    """When every polygon is a rectangle its four edges are its box sides, so
    the full-edge track returns what the box track returns."""
    rng = np.random.default_rng(5)
    n_bits = 0
    for _ in range(60):
        rects = separated_rectangles(rng, 40, int(rng.integers(1, 5)))
        jit = [(x0 + int(rng.integers(-1, 2)), x1 + int(rng.integers(-1, 2)),
                y0 + int(rng.integers(-1, 2)), y1 + int(rng.integers(-1, 2))) for x0, x1, y0, y1 in rects]
        jit = [(x0, max(x0 + 1, x1), y0, max(y0 + 1, y1)) for x0, x1, y0, y1 in jit]
        ty, tx = int(rng.integers(-3, 4)), int(rng.integers(-3, 4))
        a_rep = raster.rasterize(rects, 40)
        a_mem = raster.rasterize([(x0 + tx, x1 + tx, y0 + ty, y1 + ty) for x0, x1, y0, y1 in jit], 40)
        if (raster.components(a_mem)[1].shape[0] != len(jit)
                or raster.components(a_rep)[1].shape[0] != len(rects)):
            continue  # jitter joined two rectangles
        for t in (0, 1, 2):
            got = contour.align(a_mem, a_rep, 4, t)
            want = edge.align(a_mem, a_rep, 4, t)
            assert (got["s"], got["E"], got["bit"], got["ok"]) == (want["s"], want["E"], want["bit"], want["ok"])
            n_bits += got["bit"]
    assert n_bits > 20


def test_differing_topology_has_no_correspondence():
    a_rep = raster.rasterize([(2, 10, 2, 10)], 16)                    # square
    a_mem = raster.rasterize([(2, 10, 2, 10), (10, 12, 2, 4)], 16)    # square with a tab
    got = contour.align(a_mem, a_rep, 4, 8)
    assert got["E"] == contour.NO_MATCH and not got["bit"] and not got["topo"]
    assert edge.align(a_mem, a_rep, 4, 8)["bit"]  # the box track accepts it


def test_envelope_cap():
    N = 64
    comb = np.zeros((N, N), bool)
    comb[0, :] = True
    comb[:, ::2] = True        # 32 teeth: one polygon with many edges
    lab, boxes, polys = contour.clip_polygons(comb)
    n_edges = sum(len(c) for p in polys for c in p)
    assert boxes.shape[0] == 1 and 120 < n_edges <= contour.MAX_EDGES
    dots = np.zeros((N, N), bool)
    dots[::2, ::2] = True      # 1024 single-pixel polygons: over the cap
    assert contour.clip_polygons(dots)[2] is None
    got = contour.align(dots, dots, 4, 4)
    assert got["s"] == (0, 0) and got["E"] == contour.NO_MATCH


# ------------------------------------------------------------ pre-filter


def low_jitter_set(seed=3, n=48, N=64):
    """Few templates, 1 px jitter: many pairs meet the full-edge constraint."""
    rng = np.random.default_rng(seed)
    tpl = clipgen.make_templates(rng, 8, N, 3, 10)
    return clipgen.make_clips(rng, tpl, N, n, 1, 4)


def test_prefilter_keeps_every_covering_pair():
    cs = low_jitter_set()
    rep, mem = clipgen.all_pairs(cs.n)
    data = [contour.clip_polygons(raster.clip_raster(cs, i)) for i in range(cs.n)]
    n_cov = n_pass = 0
    for t in (1, 3):
        for r, m in zip(rep.tolist(), mem.tolist()):
            ok = contour.pair_pass(data[r], data[m], t)
            n_pass += ok
            for mm, rr in ((m, r), (r, m)):
                res = contour.align(raster.clip_raster(cs, mm), raster.clip_raster(cs, rr), int(cs.marker_w[mm]), t,
                                    data[mm], data[rr])
                if res["bit"]:
                    n_cov += 1
                    assert ok, (r, m, t)
    assert n_cov >= 40 and n_pass < 2 * rep.size * 0.5


def test_contour_results_through_cover_driver():
    cs = clipgen.small(n_clips=24)
    rep, mem = clipgen.all_pairs(cs.n)
    res = cover.align_pairs_contour(cs, rep, mem, 2)
    for k in range(0, rep.size, 17):
        for d, (m, r) in enumerate(((mem[k], rep[k]), (rep[k], mem[k]))):
            want = contour.align(raster.clip_raster(cs, m), raster.clip_raster(cs, r), int(cs.marker_w[m]), 2)
            assert tuple(res["shift"][k, d]) == want["s"] and res["E"][k, d] == want["E"]
            assert bool((res["bits"][k] >> d) & 1) == want["bit"]
