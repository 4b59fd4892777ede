"""Pair-list drivers for the oracle: per-pair alignment results and clusters.

An unordered candidate pair is given as (rep[k], mem[k]).  Both directions
are evaluated, each by the plain per-direction definition:

* direction 0: member mem[k] aligned to representative rep[k]
  -> bit0 = "rep[k] covers mem[k]", shift[k, 0] = member displacement;
* direction 1: member rep[k] aligned to representative mem[k]
  -> bit1 = "mem[k] covers rep[k]", shift[k, 1].

Pairs of clips with different raster sizes are never comparable (different
pattern radii give incomparable windows).
"""
from __future__ import annotations

import multiprocessing as mp
import os
from fractions import Fraction

import numpy as np

from . import contour, cosine, edge, loop, raster, xcorr, xysep

_SHARED = {}


class Prepared:
    """Per-clip rasters, pixel counts and whitened FP64 spectra (lazy)."""

    def __init__(self, clips):
        self.clips = clips
        self._a, self._W, self._P = {}, {}, {}

    def a(self, i):
        i = int(i)
        if i not in self._a:
            self._a[i] = raster.clip_raster(self.clips, i)
        return self._a[i]

    def W(self, i):
        i = int(i)
        if i not in self._W:
            self._W[i] = cosine.whiten(cosine.spectrum(self.a(i)))
        return self._W[i]

    def w(self, i):
        return int(self.clips.marker_w[int(i)])

    def polys(self, i):
        """Labels, boxes and full-edge polygons (`contour.clip_polygons`)."""
        i = int(i)
        if i not in self._P:
            self._P[i] = contour.clip_polygons(self.a(i))
        return self._P[i]


def _cosine_chunk(args):
    rep, mem, p, q = args
    prep = _SHARED["prep"]
    n = rep.size
    bits = np.zeros(n, np.uint8)
    shift = np.zeros((n, 2, 2), np.int16)
    c = np.zeros((n, 2), np.int32)
    sc = np.zeros((n, 2), np.float64)
    r1 = np.zeros((n, 2), np.float64)
    for k in range(n):
        j, i = int(rep[k]), int(mem[k])
        for d, (m, r) in enumerate(((i, j), (j, i))):
            res = cosine.align(prep.a(m), prep.a(r), prep.W(m), prep.W(r), prep.w(m), p, q)
            bits[k] |= np.uint8(res["bit"]) << d
            shift[k, d] = res["s"]
            c[k, d] = res["c"]
            sc[k, d] = res["score"]
            r1[k, d] = res["r1"]
    return bits, shift, c, sc, r1


def _xcorr_chunk(args):
    rep, mem, p, q = args
    prep = _SHARED["prep"]
    n = rep.size
    bits = np.zeros(n, np.uint8)
    shift = np.zeros((n, 2, 2), np.int16)
    c = np.zeros((n, 2), np.int32)
    sc = np.zeros((n, 2), np.float64)
    for k in range(n):
        j, i = int(rep[k]), int(mem[k])
        for d, (m, r) in enumerate(((i, j), (j, i))):
            res = xcorr.align(prep.a(m), prep.a(r), prep.w(m), p, q)
            bits[k] |= np.uint8(res["bit"]) << d
            shift[k, d] = res["s"]
            c[k, d] = res["c"]
            sc[k, d] = res["score"]
    return bits, shift, c, sc


def _xysep_chunk(args):
    rep, mem, p, q = args
    prep = _SHARED["prep"]
    n = rep.size
    bits = np.zeros(n, np.uint8)
    shift = np.zeros((n, 2, 2), np.int16)
    c = np.zeros((n, 2), np.int32)
    sc = np.zeros((n, 2), np.float64)
    matched = np.zeros((n, 2), bool)
    for k in range(n):
        j, i = int(rep[k]), int(mem[k])
        for d, (m, r) in enumerate(((i, j), (j, i))):
            res = xysep.align(prep.a(m), prep.a(r), prep.w(m), p, q)
            bits[k] |= np.uint8(res["bit"]) << d
            shift[k, d] = res["s"]
            c[k, d] = res["c"]
            sc[k, d] = res["score"]
            matched[k, d] = res["matched"]
    return bits, shift, c, sc, matched


def _edge_chunk(args):
    rep, mem, t_edge = args
    prep = _SHARED["prep"]
    n = rep.size
    bits = np.zeros(n, np.uint8)
    shift = np.zeros((n, 2, 2), np.int16)
    E = np.zeros((n, 2), np.int32)
    ok = np.zeros((n, 2), bool)
    for k in range(n):
        j, i = int(rep[k]), int(mem[k])
        for d, (m, r) in enumerate(((i, j), (j, i))):
            res = edge.align(prep.a(m), prep.a(r), prep.w(m), t_edge)
            bits[k] |= np.uint8(res["bit"]) << d
            shift[k, d] = res["s"]
            E[k, d] = res["E"]
            ok[k, d] = res["ok"]
    return bits, shift, E, ok


def _contour_chunk(args):
    rep, mem, t_edge = args
    prep = _SHARED["prep"]
    n = rep.size
    bits = np.zeros(n, np.uint8)
    shift = np.zeros((n, 2, 2), np.int16)
    E = np.zeros((n, 2), np.int32)
    ok = np.zeros((n, 2), bool)
    topo = np.zeros((n, 2), bool)
    for k in range(n):
        j, i = int(rep[k]), int(mem[k])
        for d, (m, r) in enumerate(((i, j), (j, i))):
            res = contour.align(prep.a(m), prep.a(r), prep.w(m), t_edge, prep.polys(m), prep.polys(r))
            bits[k] |= np.uint8(res["bit"]) << d
            shift[k, d] = res["s"]
            E[k, d] = res["E"]
            ok[k, d] = res["ok"]
            topo[k, d] = res["topo"]
    return bits, shift, E, ok, topo


def _run(fn, clips, rep, mem, extra, workers):
    rep = np.asarray(rep, np.int64)
    mem = np.asarray(mem, np.int64)
    if np.any(clips.raster_n[rep] != clips.raster_n[mem]):
        raise ValueError("pairs must have equal raster sizes")
    _SHARED["prep"] = Prepared(clips)
    workers = workers or 1
    if workers == 1 or rep.size < 64:
        parts = [fn((rep, mem) + extra)]
    else:
        chunks = np.array_split(np.arange(rep.size), workers * 4)
        ctx = mp.get_context("fork")
        with ctx.Pool(workers) as pool:
            parts = pool.map(fn, [(rep[c], mem[c]) + extra for c in chunks])
    return [np.concatenate([p[t] for p in parts]) for t in range(len(parts[0]))]


def align_pairs_cosine(clips, rep, mem, p, q, workers=None):
    """Cosine track on a pair list: dict(bits, shift, c, score, r1)."""
    bits, shift, c, sc, r1 = _run(_cosine_chunk, clips, rep, mem, (p, q), workers)
    return dict(bits=bits, shift=shift, c=c, score=sc, r1=r1)


def align_pairs_xcorr(clips, rep, mem, p, q, workers=None):
    """Exact-objective alignment on a pair list: dict(bits, shift, c, score)."""
    bits, shift, c, sc = _run(_xcorr_chunk, clips, rep, mem, (p, q), workers)
    return dict(bits=bits, shift=shift, c=c, score=sc)


def align_pairs_xysep(clips, rep, mem, p, q, workers=None):
    """Cosine track aligned by XY separation (Sec. 3.2.1(2)):
    dict(bits, shift, c, score, matched)."""
    bits, shift, c, sc, matched = _run(_xysep_chunk, clips, rep, mem, (p, q), workers)
    return dict(bits=bits, shift=shift, c=c, score=sc, matched=matched)


def align_pairs_edge(clips, rep, mem, t_edge, workers=None):
    """Edge track on a pair list: dict(bits, shift, E, ok)."""
    bits, shift, E, ok = _run(_edge_chunk, clips, rep, mem, (t_edge,), workers)
    return dict(bits=bits, shift=shift, E=E, ok=ok)


def align_pairs_contour(clips, rep, mem, t_edge, workers=None):
    """Edge track over full boundary edges (`contour`) on a pair list:
    dict(bits, shift, E, ok, topo)."""
    bits, shift, E, ok, topo = _run(_contour_chunk, clips, rep, mem, (t_edge,), workers)
    return dict(bits=bits, shift=shift, E=E, ok=ok, topo=topo)


def pixel_counts(clips):
    return np.array([int(raster.clip_raster(clips, i).sum()) for i in range(clips.n)], np.int64)


def cluster_cosine(clips, p, q, K=1, rep=None, mem=None, res=None, workers=None, relax=Fraction(2, 100)):
    """Closed loop on the cosine track over a candidate pair list (default: all
    same-size pairs), with the schedule's total relaxation `relax`.  Returns
    dict(rep_of, shift, n_clusters, reps, log)."""
    n = clips.n
    if rep is None:
        from clipgen import same_size_pairs
        rep, mem = same_size_pairs(clips)
    if res is None:
        res = align_pairs_cosine(clips, rep, mem, p, q, workers)
    cnt = pixel_counts(clips)
    rep = np.asarray(rep, np.int64)
    mem = np.asarray(mem, np.int64)

    def bits_at(tau):
        pt, qt = tau
        cov = np.zeros((n, n), bool)
        np.fill_diagonal(cov, True)
        for d, (r_, m_) in enumerate(((rep, mem), (mem, rep))):
            c = res["c"][:, d].astype(object)
            nm, nr = cnt[m_].astype(object), cnt[r_].astype(object)
            ok = (nm > 0) & (nr > 0) & (c * c * qt * qt > pt * pt * nm * nr)
            ok = ok.astype(bool)
            cov[r_[ok], m_[ok]] = True
        return cov

    sched = loop.cosine_schedule(p, q, K, relax)
    rep_of, reps, log = loop.run(n, bits_at, sched)
    return dict(rep_of=rep_of, shift=_center_shift(n, rep, mem, res["shift"], rep_of),
                n_clusters=len(reps), reps=reps, log=log)


def cluster_edge(clips, t_edge, K=1, rep=None, mem=None, res=None, workers=None, step=1, edges="box"):
    """Closed loop on the edge track (see cluster_cosine), `step` pixels of
    relaxation per coarse iteration; `edges` names the corresponding edges:
    "box" (bounding-box sides, `edge`) or "contour" (full boundary edges)."""
    n = clips.n
    if rep is None:
        from clipgen import same_size_pairs
        rep, mem = same_size_pairs(clips)
    if res is None:
        fn = align_pairs_contour if edges == "contour" else align_pairs_edge
        res = fn(clips, rep, mem, t_edge, workers)
    rep = np.asarray(rep, np.int64)
    mem = np.asarray(mem, np.int64)

    def bits_at(tau):
        cov = np.zeros((n, n), bool)
        np.fill_diagonal(cov, True)
        for d, (r_, m_) in enumerate(((rep, mem), (mem, rep))):
            ok = res["ok"][:, d] & (res["E"][:, d] >= 0) & (res["E"][:, d] <= tau)
            cov[r_[ok], m_[ok]] = True
        return cov

    sched = loop.edge_schedule(t_edge, K, step)
    rep_of, reps, log = loop.run(n, bits_at, sched)
    return dict(rep_of=rep_of, shift=_center_shift(n, rep, mem, res["shift"], rep_of),
                n_clusters=len(reps), reps=reps, log=log)


def _center_shift(n, rep, mem, shift, rep_of):
    """Each node's shift relative to its representative (0 for representatives)."""
    out = np.zeros((n, 2), np.int16)
    lookup = {}
    for k in range(rep.size):
        lookup[(int(rep[k]), int(mem[k]))] = shift[k, 0]
        lookup[(int(mem[k]), int(rep[k]))] = shift[k, 1]
    for i in range(n):
        r = int(rep_of[i])
        if r != i:
            out[i] = lookup[(r, i)]
    return out


def default_workers():
    return max(1, len(os.sched_getaffinity(0)))


def cover_csr(n, rep, mem, bits, shift, value, score):
    """The directed cover relation (Sec. 3.1 stage 2, the sparse similarity
    graph) from per-pair results of both directions: an entry (r, m) for every
    set bit, "r covers m", with m's shift relative to r, the count or residual
    and the score.  Rows r ascending, members ascending within a row; the
    diagonal (every clip covers itself) is left implicit.  Returns dict of
    row_ptr int64[n+1], col int32, shift int16[:, 2], value int32, score f64."""
    rows = [[] for _ in range(n)]
    for k in range(len(rep)):
        for d, (r, m) in enumerate(((int(rep[k]), int(mem[k])), (int(mem[k]), int(rep[k])))):
            if (int(bits[k]) >> d) & 1:
                rows[r].append((m, int(shift[k][d][0]), int(shift[k][d][1]), int(value[k][d]), float(score[k][d])))
    row_ptr = np.zeros(n + 1, np.int64)
    ent = []
    for r in range(n):
        row = sorted(rows[r])
        ent += row
        row_ptr[r + 1] = row_ptr[r] + len(row)
    return dict(row_ptr=row_ptr,
                col=np.array([e[0] for e in ent], np.int32),
                shift=np.array([(e[1], e[2]) for e in ent], np.int16).reshape(-1, 2),
                value=np.array([e[3] for e in ent], np.int32),
                score=np.array([e[4] for e in ent], np.float64))


def verify_centers(clips, rep_of, center_shift, kind, thr):
    """Center validity and cluster consistency (Sec. 2.3) of an assignment:
    the list of clips that violate it.  A representative represents itself
    with shift (0, 0); every other clip i with representative r = rep_of[i]
    must meet the constraint at its center against r:
    cosine (thr = (p, q)): the shift is a residue of i's window (C0 rule) and
    Eq. 2 holds for the overlap count at it;
    edge (thr = T): the shift lies in i's window, at it the fewer side's
    polygons (both sides if equal) each overlap exactly one polygon of the
    other clip, and over the matched bounding-box edges max |d - s| <= T;
    contour (thr = T): as edge, over the full boundary edges of the matched
    polygons, whose descriptors must be equal (`contour.residual_at`)."""
    bad = []
    n = clips.n
    for i in range(n):
        r = int(rep_of[i])
        dy, dx = int(center_shift[i][0]), int(center_shift[i][1])
        if r < 0 or r >= n:
            bad.append(i)
            continue
        if r == i:
            if dy or dx:
                bad.append(i)
            continue
        if int(rep_of[r]) != r or clips.raster_n[i] != clips.raster_n[r]:
            bad.append(i)
            continue
        a_m, a_r = raster.clip_raster(clips, i), raster.clip_raster(clips, r)
        w, N = int(clips.marker_w[i]), int(clips.raster_n[i])
        if kind == "cosine":
            axis = cosine.window_axis(w, N)
            ok = dy in axis and dx in axis
            if ok:
                c = cosine.overlap(a_r, a_m, dy, dx)
                ok = cosine.bit(c, int(a_m.sum()), int(a_r.sum()), thr[0], thr[1])
        elif kind == "contour":
            ok = abs(dy) <= w and abs(dx) <= w
            if ok:
                E = contour.residual_at(a_m, a_r, dy, dx)
                ok = E is not None and E <= thr
        else:
            ok = abs(dy) <= w and abs(dx) <= w
            if ok:
                lab_m, box_m = raster.components(a_m)
                lab_r, box_r = raster.components(a_r)
                Pm, Pr = box_m.shape[0], box_r.shape[0]
                pairs = None
                if Pm and Pr:
                    pairs = edge.correspondence(edge.overlap_relation(lab_m, lab_r, Pm, Pr, dy, dx), Pm, Pr)
                ok = pairs is not None
                if ok:
                    E = 0
                    for p_, q_ in pairs:
                        bm, br = box_m[p_ - 1], box_r[q_ - 1]
                        E = max(E, abs(int(bm[0] - br[0]) - dx), abs(int(bm[1] - br[1]) - dx),
                                abs(int(bm[2] - br[2]) - dy), abs(int(bm[3] - br[3]) - dy))
                    ok = E <= thr
        if not ok:
            bad.append(i)
    return bad
