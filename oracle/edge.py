"""Edge track: polygon correspondence and Min-Max alignment (FP64 / exact int).

Follows paper Sec. 2.2.2 (edge movement constraint: for the pattern with
fewer polygons each polygon must overlap exactly one polygon of the other
pattern, and corresponding edges may move at most T_edge) and Sec. 3.2.2,
Eq. 6 (T_opt = argmin_T max_i |d_i - T|_inf, solved per axis by the midpoint
of [d_min, d_max], residual E = (d_max - d_min)/2).

Readings fixed here:

* Polygons are 4-connected raster components; the corresponding edges of a
  matched polygon pair are the four sides of their bounding boxes, and the
  displacement of an edge is member edge minus representative edge.
* Overlap at shift s is linear (zero fill, no wrap): member polygon p
  overlaps representative polygon q iff some representative pixel x in q has
  member pixel x + s in p.
* Shifts are integers.  Per axis s = clamp(round-half-toward-zero((d_min +
  d_max)/2), -w, w); the residual is max(d_max - s, s - d_min) and
  E = max(E_x, E_y).  This equals the integer argmin of the residual with
  ties to the smaller |s|, restricted to the member's window.
* With equal polygon counts the exactly-one rule must hold from both sides.
* The correspondence is taken at T0, the Min-Max solve of the two clips'
  global bounding boxes, then re-checked at the final shift: the matching
  must be unchanged.  "Must not exceed" means E <= T_edge.
* A clip without polygons covers only itself.
"""
from __future__ import annotations

import numpy as np

from . import raster

NO_MATCH = -1  # E reported when no valid correspondence exists


def round_half_toward_zero_half(m2: int) -> int:
    """round-half-toward-zero(m2 / 2) for an integer m2, exactly."""
    return m2 // 2 if m2 >= 0 else -((-m2) // 2)


def minmax_1d(ds, w: int):
    """1-D Min-Max (Eq. 6 per axis): (s, E) for displacements ds, |s| <= w."""
    lo, hi = int(min(ds)), int(max(ds))
    s = round_half_toward_zero_half(lo + hi)
    s = max(-w, min(w, s))
    return s, max(hi - s, s - lo)


def overlap_relation(lab_mem, lab_rep, Pm, Pr, dy, dx):
    """Boolean [Pm+1, Pr+1] matrix: rel[p, q] iff member p overlaps rep q at s."""
    N = lab_rep.shape[0]
    rel = np.zeros((Pm + 1, Pr + 1), dtype=bool)
    y0, y1 = max(0, -dy), min(N, N - dy)
    x0, x1 = max(0, -dx), min(N, N - dx)
    if y0 >= y1 or x0 >= x1:
        return rel
    rep = lab_rep[y0:y1, x0:x1]
    mem = lab_mem[y0 + dy:y1 + dy, x0 + dx:x1 + dx]
    both = (rep > 0) & (mem > 0)
    rel[mem[both], rep[both]] = True
    return rel


def correspondence(rel, Pm, Pr):
    """Exactly-one overlap rule from the fewer side (both if equal).

    Returns the sorted list of matched (p, q) pairs, or None if it fails.
    """
    pairs = set()
    if Pm <= Pr:
        for p in range(1, Pm + 1):
            qs = np.flatnonzero(rel[p, 1:]) + 1
            if qs.size != 1:
                return None
            pairs.add((p, int(qs[0])))
    if Pr <= Pm:
        for q in range(1, Pr + 1):
            ps = np.flatnonzero(rel[1:, q]) + 1
            if ps.size != 1:
                return None
            pairs.add((int(ps[0]), q))
    return sorted(pairs)


def solve(box_mem, box_rep, pairs, w):
    """Min-Max over the bounding-box edges of matched pairs: (sy, sx, E)."""
    dxs, dys = [], []
    for p, q in pairs:
        bm, br = box_mem[p - 1], box_rep[q - 1]
        dxs += [int(bm[0] - br[0]), int(bm[1] - br[1])]
        dys += [int(bm[2] - br[2]), int(bm[3] - br[3])]
    sx, ex = minmax_1d(dxs, w)
    sy, ey = minmax_1d(dys, w)
    return sy, sx, max(ex, ey)


def align(a_mem, a_rep, w_mem: int, t_edge: int):
    """Edge-track alignment of member to representative.

    Returns dict(s=(dy, dx), E, bit, ok) where ok says a correspondence was
    found and survived the re-check; E = NO_MATCH when none was found.
    """
    lab_m, box_m = raster.components(a_mem)
    lab_r, box_r = raster.components(a_rep)
    Pm, Pr = box_m.shape[0], box_r.shape[0]
    if Pm == 0 or Pr == 0:
        return dict(s=(0, 0), E=NO_MATCH, bit=False, ok=False)
    gm, gr = raster.global_bbox(a_mem), raster.global_bbox(a_rep)
    sy0, sx0, _ = solve(np.array([gm]), np.array([gr]), [(1, 1)], w_mem)
    pairs0 = correspondence(overlap_relation(lab_m, lab_r, Pm, Pr, sy0, sx0), Pm, Pr)
    if pairs0 is None:
        return dict(s=(sy0, sx0), E=NO_MATCH, bit=False, ok=False)
    sy, sx, E = solve(box_m, box_r, pairs0, w_mem)
    pairs1 = correspondence(overlap_relation(lab_m, lab_r, Pm, Pr, sy, sx), Pm, Pr)
    ok = pairs1 == pairs0
    return dict(s=(sy, sx), E=int(E), bit=bool(ok and E <= t_edge), ok=bool(ok))
