"""Clip model (paper Sec. 2.1, Eq. 1; cosine-track step 1 "Rasterization").

A pattern is the layout content inside a square window of the pattern radius
around its center.  In the clip model each clip is already expressed in its
own window frame: a list of half-open integer rectangles and a raster size N.
Pixel (y, x) is 1 iff some rectangle has x0 <= x < x1 and y0 <= y < y1;
content outside [0, N) is clipped away.

Polygons (Sec. 2.2.2, "Polygon Overlap") are read as the 4-connected
components of the raster, each described by its bounding box
[x0, x1) x [y0, y1).
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

FOUR_CONNECTED = np.array([[0, 1, 0], [1, 1, 1], [0, 1, 0]], dtype=bool)


def rasterize(rects, N) -> np.ndarray:
    """Binary N x N raster of a list of half-open rectangles (x0, x1, y0, y1)."""
    a = np.zeros((N, N), dtype=bool)
    for x0, x1, y0, y1 in np.asarray(rects, dtype=np.int64).reshape(-1, 4):
        x0, x1 = max(int(x0), 0), min(int(x1), N)
        y0, y1 = max(int(y0), 0), min(int(y1), N)
        if x0 < x1 and y0 < y1:
            a[y0:y1, x0:x1] = True
    return a


def clip_raster(clips, i) -> np.ndarray:
    """Raster of clip ``i`` of a ``clipgen.ClipSet``."""
    lo, hi = int(clips.rect_ptr[i]), int(clips.rect_ptr[i + 1])
    return rasterize(clips.rects[lo:hi], int(clips.raster_n[i]))


def rasters(clips, idx=None):
    idx = range(clips.n) if idx is None else idx
    return [clip_raster(clips, int(i)) for i in idx]


def components(a):
    """4-connected components: (label image int32, bboxes int64 [P, 4]).

    Labels are 1..P in raster order of each component's first pixel; the
    bounding box of label p is row p-1 as half-open (x0, x1, y0, y1).
    """
    lab, P = ndimage.label(a, structure=FOUR_CONNECTED)
    boxes = np.zeros((P, 4), dtype=np.int64)
    for p, sl in enumerate(ndimage.find_objects(lab), start=0):
        ys, xs = sl
        boxes[p] = (xs.start, xs.stop, ys.start, ys.stop)
    return lab.astype(np.int32), boxes


def global_bbox(a):
    """Half-open bounding box (x0, x1, y0, y1) of all set pixels, or None."""
    ys, xs = np.nonzero(a)
    if ys.size == 0:
        return None
    return (int(xs.min()), int(xs.max()) + 1, int(ys.min()), int(ys.max()) + 1)
