"""Full boundary-edge correspondence for the edge track, and the topological
hash pre-filter (test infrastructure, exact integers, CPU only).

Paper Sec. 2.2.2 states the edge movement constraint over corresponding edges
of matched polygons; Sec. 1.4 (item 4) and Sec. 3.1 (stage 1) name
topological hashing as a pre-screen.  `edge` reads the corresponding edges as
the four sides of each polygon's bounding box; this module uses every edge of
the polygon boundary.

Readings fixed here:

* Boundary.  The boundary of a polygon (a 4-connected component,
  `raster.components`) is made of the unit pixel sides between one of its
  pixels and a pixel outside it (outside the raster counts as outside).  A
  side is directed so that the polygon lies on its right in image
  coordinates (x to the right, y down): top sides run east, right sides
  south, bottom sides west, left sides north.  Corners are (x, y) with x, y in
  [0, N].
* Contours.  Directed sides joined end to start form closed contours.  Where
  two sides of the polygon leave the same corner (two of its pixels meet
  there only diagonally) the contour turns right, so those pixels stay apart
  as 4-connectivity has them.  An edge is a maximal run of sides in one
  direction; a vertex is the corner where an edge starts.  A polygon has one
  outer contour (four more right turns than left turns) and one contour per
  hole (four more left turns); the holes are the components of the
  polygon's complement under 8-connectivity that do not reach the border.
* Canonical start.  Directions are coded E = 0, S = 1, W = 2, N = 3.  A
  contour starts at the lexicographically least rotation of its code
  sequence.  The sequence has no shorter period (its turns add up to exactly
  one full turn, which a repetition would multiply), so the rotation is
  unique, and contours with equal cyclic sequences get equal canonical
  sequences edge for edge.
* Order.  A polygon lists its outer contour first, then its holes in raster
  order of their first vertex (least (y, x)).  Its descriptor is the tuple of
  the canonical code sequences in that order.
* Correspondence.  Polygons are matched as in `edge` (exactly-one overlap at
  T0 from the fewer side, both if equal).  Each matched pair must have equal
  descriptors, else there is no correspondence (E = NO_MATCH, shift T0);
  then edge k of the member polygon corresponds to edge k of the
  representative polygon.  A vertical edge (S, N) is displaced along x by the
  difference of the two x coordinates, a horizontal edge (E, W) along y by
  the difference of the y coordinates, member minus representative.
* The Min-Max solve, rounding, window clamp, re-check at the solved shift
  and the threshold test are those of `edge`.
* Envelope.  A clip with more than MAX_POLYGONS polygons or more than
  MAX_EDGES edges over all its polygons has no contour data: every pair
  with it (or with an empty clip) gets shift (0, 0), E = NO_MATCH.
* Topological hash.  The hash of a polygon is FNV-1a (64-bit) over the bytes
  of its descriptor (each contour's codes, then the byte 4), low 32 bits
  kept.  Pre-filter: a pair survives iff every polygon of the fewer side (both
  sides if equal) has a polygon on the other side with the same hash and
  with bounding-box width and height within 2 T_edge (bound B3).  A pair
  that meets the constraint survives: its matched polygons have equal
  descriptors, and the extreme vertical (horizontal) edges of the two
  polygons force a spread of at least the width (height) difference among
  the displacements, so the residual is at least half of it.
"""
from __future__ import annotations

import numpy as np

from . import edge, raster

NO_MATCH = edge.NO_MATCH
MAX_POLYGONS = 64
MAX_EDGES = 4096          # edges over all polygons of one clip
E_, S_, W_, N_ = 0, 1, 2, 3
STEP = {E_: (1, 0), S_: (0, 1), W_: (-1, 0), N_: (0, -1)}  # (dx, dy) along a direction
FNV_OFFSET = 0xCBF29CE484222325
FNV_PRIME = 0x100000001B3


def sides(inside):
    """Directed unit sides of a boolean mask, as {start corner (x, y): [directions]}."""
    H, W = inside.shape
    pad = np.zeros((H + 2, W + 2), dtype=bool)
    pad[1:-1, 1:-1] = inside
    out = {}
    ys, xs = np.nonzero(inside)
    for y, x in zip(ys.tolist(), xs.tolist()):
        if not pad[y, x + 1]:          # above is outside: top side, east
            out.setdefault((x, y), []).append(E_)
        if not pad[y + 1, x + 2]:      # right is outside: right side, south
            out.setdefault((x + 1, y), []).append(S_)
        if not pad[y + 2, x + 1]:      # below is outside: bottom side, west
            out.setdefault((x + 1, y + 1), []).append(W_)
        if not pad[y + 1, x]:          # left is outside: left side, north
            out.setdefault((x, y + 1), []).append(N_)
    return out


def contours(inside):
    """Closed contours of a mask, each a list of edges (direction, x, y) with
    (x, y) the edge's start vertex, in traversal order from the contour's
    raster-first corner."""
    out = sides(inside)
    remaining = {(c, d) for c, ds in out.items() for d in ds}
    result = []
    while remaining:
        start = min(remaining, key=lambda cd: (cd[0][1], cd[0][0], cd[1]))
        steps = []
        c, d = start
        while True:
            remaining.discard((c, d))
            steps.append((d, c))
            nxt = (c[0] + STEP[d][0], c[1] + STEP[d][1])
            cand = out[nxt]
            if len(cand) == 1:
                nd = cand[0]
            else:
                nd = (d + 1) % 4          # two ways out: turn right
                assert nd in cand
            c, d = nxt, nd
            if (c, d) == start:
                break
        # the raster-first corner is a turn, so steps[0] starts an edge
        edges = []
        for k, (d, c) in enumerate(steps):
            if k == 0 or d != steps[k - 1][0]:
                edges.append((d, c[0], c[1]))
        result.append(edges)
    return result


def turning(edges):
    """Right turns minus left turns around a closed contour."""
    t = 0
    for k in range(len(edges)):
        d, d2 = edges[k][0], edges[(k + 1) % len(edges)][0]
        t += 1 if d2 == (d + 1) % 4 else -1
    return t


def least_rotation(codes):
    """Start index of the lexicographically least rotation (unique)."""
    codes = tuple(codes)
    n = len(codes)

    def rot(i):
        return codes[i:] + codes[:i]

    best = min(range(n), key=rot)
    least = rot(best)
    assert sum(1 for i in range(n) if rot(i) == least) == 1, "direction sequence with a shorter period"
    return best


def coord(e):
    """The coordinate an edge is displaced along: x for S/N, y for E/W."""
    d, x, y = e
    return x if d in (S_, N_) else y


def polygon(inside):
    """Edges of one polygon in its canonical order: list of contours, each a
    list of (direction, coordinate); contour 0 is the outer one."""
    return canonical(contours(inside))


def canonical(cons):
    """The contours of one polygon in canonical order (see `polygon`)."""
    outer = [c for c in cons if turning(c) == 4]
    holes = [c for c in cons if turning(c) == -4]
    assert len(outer) == 1 and len(outer) + len(holes) == len(cons)
    holes.sort(key=lambda c: min((y, x) for _, x, y in c))
    out = []
    for c in outer + holes:
        r = least_rotation([e[0] for e in c])
        c = c[r:] + c[:r]
        out.append([(e[0], coord(e)) for e in c])
    return out


def descriptor(poly):
    return tuple(tuple(d for d, _ in c) for c in poly)


def fnv1a64(data: bytes) -> int:
    """FNV-1a, 64-bit (Fowler, Noll, Vo): per byte, xor then multiply."""
    h = FNV_OFFSET
    for b in data:
        h ^= b
        h = (h * FNV_PRIME) & 0xFFFFFFFFFFFFFFFF
    return h


def poly_hash(poly) -> int:
    data = bytearray()
    for c in poly:
        data += bytes(d for d, _ in c)
        data.append(4)
    return fnv1a64(bytes(data)) & 0xFFFFFFFF


def clip_polygons(a):
    """(labels, boxes, polygons) of a raster; polygons is None outside the
    envelope (more than MAX_POLYGONS polygons or MAX_EDGES edges)."""
    lab, boxes = raster.components(a)
    P = boxes.shape[0]
    if P > MAX_POLYGONS:
        return lab, boxes, None
    cons = [contours(lab == p) for p in range(1, P + 1)]
    if sum(len(c) for cc in cons for c in cc) > MAX_EDGES:
        return lab, boxes, None
    return lab, boxes, [canonical(cc) for cc in cons]


def solve(polys_m, polys_r, pairs, w):
    """Min-Max over the corresponding edges of matched pairs: (sy, sx, E), or
    None when a matched pair has different descriptors."""
    dxs, dys = [], []
    for p, q in pairs:
        pm, pr = polys_m[p - 1], polys_r[q - 1]
        if descriptor(pm) != descriptor(pr):
            return None
        for cm, cr in zip(pm, pr):
            for (d, um), (_, ur) in zip(cm, cr):
                (dxs if d in (S_, N_) else dys).append(um - ur)
    sx, ex = edge.minmax_1d(dxs, w)
    sy, ey = edge.minmax_1d(dys, w)
    return sy, sx, max(ex, ey)


def align(a_mem, a_rep, w_mem: int, t_edge: int, data_mem=None, data_rep=None):
    """Edge-track alignment of member to representative over full boundary
    edges.  Returns dict(s=(dy, dx), E, bit, ok, topo) where ok says a
    correspondence was found, had equal descriptors and survived the re-check,
    and topo says the matched descriptors were equal."""
    lab_m, box_m, polys_m = data_mem if data_mem is not None else clip_polygons(a_mem)
    lab_r, box_r, polys_r = data_rep if data_rep is not None else clip_polygons(a_rep)
    Pm, Pr = box_m.shape[0], box_r.shape[0]
    if Pm == 0 or Pr == 0 or polys_m is None or polys_r is None:
        return dict(s=(0, 0), E=NO_MATCH, bit=False, ok=False, topo=False)
    gm, gr = raster.global_bbox(a_mem), raster.global_bbox(a_rep)
    sy0, sx0, _ = edge.solve(np.array([gm]), np.array([gr]), [(1, 1)], w_mem)
    pairs0 = edge.correspondence(edge.overlap_relation(lab_m, lab_r, Pm, Pr, sy0, sx0), Pm, Pr)
    if pairs0 is None:
        return dict(s=(sy0, sx0), E=NO_MATCH, bit=False, ok=False, topo=False)
    sol = solve(polys_m, polys_r, pairs0, w_mem)
    if sol is None:
        return dict(s=(sy0, sx0), E=NO_MATCH, bit=False, ok=False, topo=False)
    sy, sx, E = sol
    pairs1 = edge.correspondence(edge.overlap_relation(lab_m, lab_r, Pm, Pr, sy, sx), Pm, Pr)
    ok = pairs1 == pairs0
    return dict(s=(sy, sx), E=int(E), bit=bool(ok and E <= t_edge), ok=bool(ok), topo=True)


def residual_at(a_mem, a_rep, dy: int, dx: int):
    """Center check at a given shift: the largest |d - s| over the corresponding
    edges of the correspondence at (dy, dx), or None when there is none
    (no polygon, outside the envelope, exactly-one fails, descriptors differ)."""
    lab_m, box_m, polys_m = clip_polygons(a_mem)
    lab_r, box_r, polys_r = clip_polygons(a_rep)
    Pm, Pr = box_m.shape[0], box_r.shape[0]
    if Pm == 0 or Pr == 0 or polys_m is None or polys_r is None:
        return None
    pairs = edge.correspondence(edge.overlap_relation(lab_m, lab_r, Pm, Pr, dy, dx), Pm, Pr)
    if pairs is None:
        return None
    E = 0
    for p, q in pairs:
        pm, pr = polys_m[p - 1], polys_r[q - 1]
        if descriptor(pm) != descriptor(pr):
            return None
        for cm, cr in zip(pm, pr):
            for (d, um), (_, ur) in zip(cm, cr):
                E = max(E, abs(um - ur - (dx if d in (S_, N_) else dy)))
    return E


def pair_pass(data_a, data_b, t_edge: int) -> bool:
    """The pre-filter on one unordered pair: topological hash plus box sizes."""
    _, box_a, polys_a = data_a
    _, box_b, polys_b = data_b
    Pa, Pb = box_a.shape[0], box_b.shape[0]
    if Pa == 0 or Pb == 0 or polys_a is None or polys_b is None:
        return False
    ha = np.array([poly_hash(p) for p in polys_a], dtype=np.int64)
    hb = np.array([poly_hash(p) for p in polys_b], dtype=np.int64)
    wa, hta = box_a[:, 1] - box_a[:, 0], box_a[:, 3] - box_a[:, 2]
    wb, htb = box_b[:, 1] - box_b[:, 0], box_b[:, 3] - box_b[:, 2]
    ok = (np.abs(wa[:, None] - wb[None, :]) <= 2 * t_edge) & \
         (np.abs(hta[:, None] - htb[None, :]) <= 2 * t_edge) & (ha[:, None] == hb[None, :])
    if Pa <= Pb and not ok.any(axis=1).all():
        return False
    if Pb <= Pa and not ok.any(axis=0).all():
        return False
    return True
