"""XY-separation Min-Max alignment for the cosine track (test infrastructure,
exact integers, CPU only).

Paper Sec. 3.2.1(2) gives a geometric alternative to phase correlation for
area (cosine) constraints, based on competition between intervals: for each
corresponding polygon pair take the allowable translation interval
[d_min, d_max] along x and along y, measure its quality Q = d_max - d_min
(a narrow interval pins the translation), pick per axis the pair with the
narrowest interval, and take that interval's midpoint as the translation on
that axis.  The cosine of Eq. 2 is then evaluated at the resulting shift.

Readings fixed here (shared with the edge track where the paper is the same):

* Polygons, their bounding boxes and their correspondence are those of the
  edge track (`edge.correspondence` at T0, the Min-Max shift of the two global
  bounding boxes): 4-connected components, exactly-one overlap from the side
  with fewer polygons (both sides if equal).
* The allowable interval of a matched pair (member polygon p, representative
  polygon q) along x is [min(d0, d1), max(d0, d1)] with d0, d1 the
  displacements (member minus representative) of its left and right box
  edges; likewise along y with the top and bottom edges.  Q is its width.
* Ties in Q go to the first matched pair in (p, q) order (polygon labels in
  raster order of their first pixel).
* The shift per axis is the interval midpoint rounded half toward zero and
  clamped to the member's window, as in the edge track; for the cosine track
  it is a circular shift, named in [-N/2, N/2 - 1] when 2 w + 1 > N.
* Without a correspondence (no polygon on a side, the exactly-one rule fails,
  or a clip has more than 64 polygons) the single pair of global bounding
  boxes is used, which gives T0.
* Score and bit are Eq. 2 at the shift (`cosine.overlap`, `cosine.score`,
  `cosine.bit`).  An empty clip gives s = (0, 0), c = 0, bit = False.
"""
from __future__ import annotations

import numpy as np

from . import cosine, edge, raster

MAX_POLYGONS = 64  # clips with more polygons have no correspondence here


def intervals(box_mem, box_rep, pairs):
    """Per matched pair (p, q): x and y intervals [lo, hi] of the box-edge
    displacements, as an int array [len(pairs), 4] (xlo, xhi, ylo, yhi)."""
    out = []
    for p, q in pairs:
        bm, br = box_mem[p - 1], box_rep[q - 1]
        d0, d1 = int(bm[0] - br[0]), int(bm[1] - br[1])
        e0, e1 = int(bm[2] - br[2]), int(bm[3] - br[3])
        out.append((min(d0, d1), max(d0, d1), min(e0, e1), max(e0, e1)))
    return np.array(out, dtype=np.int64).reshape(-1, 4)


def winner(lo, hi):
    """Index of the narrowest interval, the first one on ties."""
    widths = hi - lo
    return int(np.flatnonzero(widths == widths.min())[0])


def residue(s: int, w: int, N: int) -> int:
    """A clamped shift named as the cosine window names it (C0 rule)."""
    if 2 * w + 1 > N:
        return (s + N // 2) % N - N // 2
    return s


def shift(a_mem, a_rep, w_mem: int):
    """The XY-separation shift of member to representative: ((dy, dx), matched)
    where matched says the polygon correspondence held."""
    N = a_mem.shape[0]
    lab_m, box_m = raster.components(a_mem)
    lab_r, box_r = raster.components(a_rep)
    Pm, Pr = box_m.shape[0], box_r.shape[0]
    gm, gr = raster.global_bbox(a_mem), raster.global_bbox(a_rep)
    pairs = None
    if 0 < Pm <= MAX_POLYGONS and 0 < Pr <= MAX_POLYGONS:
        sy0, sx0, _ = edge.solve(np.array([gm]), np.array([gr]), [(1, 1)], w_mem)
        pairs = edge.correspondence(edge.overlap_relation(lab_m, lab_r, Pm, Pr, sy0, sx0), Pm, Pr)
    if pairs is None:
        iv = intervals(np.array([gm]), np.array([gr]), [(1, 1)])
    else:
        iv = intervals(box_m, box_r, pairs)
    kx = winner(iv[:, 0], iv[:, 1])
    ky = winner(iv[:, 2], iv[:, 3])
    sx, _ = edge.minmax_1d([iv[kx, 0], iv[kx, 1]], w_mem)
    sy, _ = edge.minmax_1d([iv[ky, 2], iv[ky, 3]], w_mem)
    return (residue(sy, w_mem, N), residue(sx, w_mem, N)), pairs is not None


def align(a_mem, a_rep, w_mem: int, p: int, q: int):
    """Member aligned to the fixed representative by XY separation, scored by
    Eq. 2.  Returns dict(s=(dy, dx), c, score, bit, matched)."""
    n_mem = int(np.count_nonzero(a_mem))
    n_rep = int(np.count_nonzero(a_rep))
    if n_mem == 0 or n_rep == 0:
        return dict(s=(0, 0), c=0, score=0.0, bit=False, matched=False)
    (dy, dx), matched = shift(a_mem, a_rep, w_mem)
    c = cosine.overlap(a_rep, a_mem, dy, dx)
    return dict(s=(dy, dx), c=c, score=cosine.score(c, n_mem, n_rep), bit=cosine.bit(c, n_mem, n_rep, p, q),
                matched=bool(matched))
