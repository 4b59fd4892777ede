"""The cheaper bounds the bounds pass runs ahead of B2 and B3 (paper Sec. 3.1
stage 1) are implied by them, so they only drop pairs B2 or B3 would drop:

* cosine: for every shift d, the exact signature term
  U(d) = sum_y min(r_rep[y], r_mem[(y + d) mod N]) is at most the 8-row-block
  term sum_Y min(A[Y], W[(8 Y + d) mod N]) (A the representative's block sums,
  W the member's sliding 8-row sums), which is at most the shift-group term
  sum_Y min(A[Y], max_{d' in G} W[(8 Y + d') mod N]) for the group G of d;
* edge: whenever B3 passes, the fewer side's (both if equal) largest and
  smallest polygon widths and heights lie within 2 T of the other side's.

Checked here on clip rasters and on constructed box sets that pass B3."""
import numpy as np

import clipgen
from oracle import prune, raster

GROUPS = ((-16, 0), (1, 16))  # the two shift groups of the half-window 16


def _terms(r_rep, r_mem, N=128):
    ys = np.arange(N)
    A = r_rep.reshape(N // 8, 8).sum(axis=1)
    W = sum(np.roll(r_mem, -k) for k in range(8))
    Ys = np.arange(N // 8)
    out = {}
    for d in range(-16, 17):
        exact = int(np.minimum(r_rep, r_mem[(ys + d) % N]).sum())
        coarse = int(np.minimum(A, W[(8 * Ys + d) % N]).sum())
        g = next(gr for gr in GROUPS if gr[0] <= d <= gr[1])
        M = np.max([W[(8 * Ys + e) % N] for e in range(g[0], g[1] + 1)], axis=0)
        group = int(np.minimum(A, M).sum())
        out[d] = (exact, coarse, group)
    return out


def test_cosine_group_and_block_terms_bound_the_signature_term():
    cs = clipgen.c128(n_clips=40, n_templates=4)
    R = [raster.clip_raster(cs, i) for i in range(cs.n)]
    checked = 0
    for i in range(cs.n):
        for j in range(i + 1, cs.n):
            for a_rep, a_mem in ((R[i], R[j]), (R[j], R[i])):
                for axis in (1, 0):  # row sums, then column sums
                    t = _terms(a_rep.sum(axis=axis).astype(np.int64), a_mem.sum(axis=axis).astype(np.int64))
                    for exact, coarse, group in t.values():
                        assert exact <= coarse <= group
                    checked += 1
            # the exact terms are the oracle's B2: their window maxima give its bound
            rows = _terms(R[i].sum(axis=1).astype(np.int64), R[j].sum(axis=1).astype(np.int64))
            cols = _terms(R[i].sum(axis=0).astype(np.int64), R[j].sum(axis=0).astype(np.int64))
            w = int(cs.marker_w[j])
            best = min(max(rows[d][0] for d in range(-w, w + 1)), max(cols[d][0] for d in range(-w, w + 1)))
            assert best == prune.signature_bound(R[j], R[i], w)
    assert checked == 4 * cs.n * (cs.n - 1) // 2


def _extremes_ok(X, Y, tol):
    wx, hx = X[:, 1] - X[:, 0], X[:, 3] - X[:, 2]
    wy, hy = Y[:, 1] - Y[:, 0], Y[:, 3] - Y[:, 2]
    return (wx.max() <= wy.max() + tol and wx.min() + tol >= wy.min() and
            hx.max() <= hy.max() + tol and hx.min() + tol >= hy.min())


def _extremes_pass(A, B, t):
    tol = 2 * t
    ok = True
    if len(A) <= len(B):
        ok &= _extremes_ok(A, B, tol)
    if len(B) <= len(A):
        ok &= _extremes_ok(B, A, tol)
    return ok


def test_b3_implies_the_extremes_test():
    rng = np.random.default_rng(5)
    passing = 0
    # constructed pairs: each box of X has a partner in Y within 2 t in width
    # and height, plus extra boxes of any size on the larger side
    for _ in range(3000):
        t = int(rng.integers(0, 5))
        px = int(rng.integers(1, 9))
        X = np.zeros((px, 4), np.int64)
        X[:, 1] = rng.integers(1, 60, px)
        X[:, 3] = rng.integers(1, 60, px)
        Y = X.copy()
        Y[:, 1] = np.maximum(1, X[:, 1] + rng.integers(-2 * t, 2 * t + 1, px))
        Y[:, 3] = np.maximum(1, X[:, 3] + rng.integers(-2 * t, 2 * t + 1, px))
        extra = int(rng.integers(0, 6))
        if extra:
            E = np.zeros((extra, 4), np.int64)
            E[:, 1] = rng.integers(1, 120, extra)
            E[:, 3] = rng.integers(1, 120, extra)
            Y = np.concatenate([Y, E])
        for A, B in ((X, Y), (Y, X)):
            if prune.edge_pair_pass(A, B, t):
                passing += 1
                assert _extremes_pass(A, B, t)
    # clip polygons of the density workload
    cs = clipgen.dense(n_clips=120, n_templates=12)
    boxes = [raster.components(raster.clip_raster(cs, i))[1] for i in range(cs.n)]
    for i in range(cs.n):
        for j in range(i + 1, cs.n):
            for t in (1, 3, 6):
                if prune.edge_pair_pass(boxes[i], boxes[j], t):
                    passing += 1
                    assert _extremes_pass(boxes[i], boxes[j], t)
    assert passing > 1000
