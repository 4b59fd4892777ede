"""Seeded synthetic inputs for batched clip alignment.

This module produces only *inputs*: rectangle lists in clip-frame pixel
coordinates, raster sizes, marker half-windows, candidate pair lists and
request traces.  It holds none of the method's arithmetic: no rasterisation,
no transform, no similarity, alignment or cover computation.  Both the FP64
oracle and the GPU path consume what it returns, and nothing else is shared
between them.

Workload recipes (the paper evaluates on contest layouts that are not
available; these synthetic sets stand in for them, shaped like its cases):

* ``small``   -- 256 clips of 64x64 from 16 templates of 4-12 rectangles,
  edge jitter +-3 px, pattern offset +-8 px inside a 17x17 marker window.
* ``c128``    -- 50,000 clips of 128x128 from 1,000 templates of 6-24
  rectangles, jitter +-4 px, offset +-16 px (33x33 marker window).
* ``mixed``   -- 200,000 clips, raster sizes 64/128/256 in ratio 4:3:1,
  windows +-4..+-32 px, Zipf(1.2) candidate-list lengths in [1, 4096].
* ``dense``   -- 128x128 clips from templates whose expected union density
  is drawn uniformly from [0.1, 0.6] (coverage targeted through rectangle
  sizes, not measured here).
* ``serving`` -- a library of one 128x128 representative per template and
  request batches with log-normal sizes arriving as a Poisson stream.

A rectangle is ``(x0, x1, y0, y1)``: pixel ``(y, x)`` of the clip raster is
covered iff ``x0 <= x < x1`` and ``y0 <= y < y1``.  Rectangles may reach
outside ``[0, N)``; consumers clip them.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 1000


@dataclass
class ClipSet:
    """Clips as a rectangle CSR plus per-clip raster size and marker window."""

    rect_ptr: np.ndarray  # int64 [n+1]
    rects: np.ndarray  # int32 [m, 4]  (x0, x1, y0, y1)
    raster_n: np.ndarray  # int16 [n]
    marker_w: np.ndarray  # int16 [n]
    template: np.ndarray  # int32 [n]  (bookkeeping only)
    offset: np.ndarray  # int16 [n, 2] (dy, dx) applied to the template
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.raster_n.shape[0])

    def subset(self, idx) -> "ClipSet":
        idx = np.asarray(idx, dtype=np.int64)
        counts = self.rect_ptr[idx + 1] - self.rect_ptr[idx]
        ptr = np.zeros(idx.size + 1, dtype=np.int64)
        np.cumsum(counts, out=ptr[1:])
        rows = np.concatenate(
            [np.arange(self.rect_ptr[i], self.rect_ptr[i + 1]) for i in idx]
        ) if idx.size else np.zeros(0, dtype=np.int64)
        return ClipSet(ptr, self.rects[rows].copy(), self.raster_n[idx].copy(),
                       self.marker_w[idx].copy(), self.template[idx].copy(),
                       self.offset[idx].copy(), dict(self.meta))


def _sorted_pair(rng, lo, hi, size):
    """Two distinct integers uniform in [lo, hi), returned sorted (a < b)."""
    a = rng.integers(lo, hi, size=size)
    b = rng.integers(lo, hi, size=size)
    bad = a == b
    while bad.any():
        b[bad] = rng.integers(lo, hi, size=int(bad.sum()))
        bad = a == b
    return np.minimum(a, b), np.maximum(a, b)


def make_templates(rng, n_templates, N, rect_lo, rect_hi, density=None):
    """Templates as lists of rectangles with corners uniform in [0, N).

    With ``density`` (an array of target coverages, one per template) the
    rectangle sizes are instead drawn so that the expected union coverage
    under independent placement, ``1 - exp(-sum(area) / N^2)``, matches the
    target; the actual coverage is only approximately the target.
    """
    out = []
    counts = rng.integers(rect_lo, rect_hi + 1, size=n_templates)
    for t in range(n_templates):
        k = int(counts[t])
        if density is None:
            x0, x1 = _sorted_pair(rng, 0, N, k)
            y0, y1 = _sorted_pair(rng, 0, N, k)
        else:
            total = -np.log1p(-float(density[t])) * N * N
            share = rng.dirichlet(np.ones(k)) * total
            aspect = np.exp(rng.uniform(-1.0, 1.0, size=k))
            wx = np.clip(np.rint(np.sqrt(share * aspect)), 1, N).astype(np.int64)
            wy = np.clip(np.rint(share / np.maximum(wx, 1)), 1, N).astype(np.int64)
            x0 = rng.integers(0, N - wx + 1)
            y0 = rng.integers(0, N - wy + 1)
            x1, y1 = x0 + wx, y0 + wy
        out.append(np.stack([x0, x1, y0, y1], axis=1).astype(np.int32))
    return out


def make_clips(rng, templates, N, n_clips, jitter, w, template_of=None):
    """Clips drawn from templates: per-edge jitter, then a whole-pattern offset.

    Each rectangle edge moves by a uniform integer in [-jitter, jitter]
    (``x1 >= x0 + 1`` and ``y1 >= y0 + 1`` enforced by raising the far edge),
    then the whole pattern moves by (dy, dx) uniform in [-w, w]^2.
    ``w`` may be a scalar or a per-clip array.
    """
    if template_of is None:
        template_of = rng.integers(0, len(templates), size=n_clips)
    template_of = np.asarray(template_of, dtype=np.int64)
    w_arr = np.broadcast_to(np.asarray(w, dtype=np.int64), (n_clips,))
    counts = np.array([templates[t].shape[0] for t in template_of], dtype=np.int64)
    ptr = np.zeros(n_clips + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    rects = np.concatenate([templates[t] for t in template_of]).astype(np.int64) \
        if n_clips else np.zeros((0, 4), np.int64)
    rects = rects + rng.integers(-jitter, jitter + 1, size=rects.shape)
    rects[:, 1] = np.maximum(rects[:, 1], rects[:, 0] + 1)
    rects[:, 3] = np.maximum(rects[:, 3], rects[:, 2] + 1)
    oy = rng.integers(-w_arr, w_arr + 1)
    ox = rng.integers(-w_arr, w_arr + 1)
    per_rect_clip = np.repeat(np.arange(n_clips), counts)
    rects[:, 0:2] += ox[per_rect_clip, None]
    rects[:, 2:4] += oy[per_rect_clip, None]
    return ClipSet(
        rect_ptr=ptr,
        rects=rects.astype(np.int32),
        raster_n=np.full(n_clips, N, dtype=np.int16),
        marker_w=w_arr.astype(np.int16).copy(),
        template=template_of.astype(np.int32),
        offset=np.stack([oy, ox], axis=1).astype(np.int16),
    )


def concat(sets):
    """Concatenate clip sets (template ids are kept as given)."""
    ptrs, off = [np.zeros(1, np.int64)], 0
    for s in sets:
        ptrs.append(s.rect_ptr[1:] + off)
        off += int(s.rect_ptr[-1])
    return ClipSet(
        rect_ptr=np.concatenate(ptrs),
        rects=np.concatenate([s.rects for s in sets]),
        raster_n=np.concatenate([s.raster_n for s in sets]),
        marker_w=np.concatenate([s.marker_w for s in sets]),
        template=np.concatenate([s.template for s in sets]),
        offset=np.concatenate([s.offset for s in sets]),
    )


# --------------------------------------------------------------------------
# Named workloads.  Every one is a pure function of (sizes, seed).


def small(seed=SEED_BASE + 1, n_clips=256, N=64, n_templates=16, jitter=3, w=8):
    """256 clips of 64x64, 16 templates of 4-12 rectangles, +-3 jitter, +-8 offset."""
    rng = np.random.default_rng(seed)
    tpl = make_templates(rng, n_templates, N, 4, 12)
    cs = make_clips(rng, tpl, N, n_clips, jitter, w)
    cs.meta.update(name="small", seed=seed, cos_p=19, cos_q=20, edge_tol=2)
    return cs


def c128(seed=SEED_BASE + 2, n_clips=50_000, n_templates=1_000, N=128, jitter=4, w=16):
    """128x128 clips from templates of 6-24 rectangles, +-4 jitter, +-16 offset."""
    rng = np.random.default_rng(seed)
    tpl = make_templates(rng, n_templates, N, 6, 24)
    cs = make_clips(rng, tpl, N, n_clips, jitter, w)
    cs.meta.update(name="c128", seed=seed, cos_p=19, cos_q=20, edge_tol=3)
    return cs


def dense(seed=SEED_BASE + 4, n_clips=2_000_000, n_templates=20_000, N=128, jitter=4, w=16):
    """128x128 clips whose templates target union density U(0.1, 0.6)."""
    rng = np.random.default_rng(seed)
    dens = rng.uniform(0.1, 0.6, size=n_templates)
    tpl = make_templates(rng, n_templates, N, 6, 24, density=dens)
    # clips per template as equal as possible, in random order
    tof = np.resize(np.arange(n_templates), n_clips)
    rng.shuffle(tof)
    cs = make_clips(rng, tpl, N, n_clips, jitter, w, template_of=tof)
    cs.meta.update(name="dense", seed=seed, cos_p=19, cos_q=20, edge_tol=2,
                   template_density=dens)
    return cs


def zipf_lengths(rng, n, s=1.2, lo=1, hi=4096):
    """List lengths ~ Zipf(s) truncated to [lo, hi] (exact inverse-CDF sampling)."""
    k = np.arange(lo, hi + 1, dtype=np.float64)
    pmf = k ** (-s)
    cdf = np.cumsum(pmf)
    cdf /= cdf[-1]
    u = rng.random(n)
    return (np.searchsorted(cdf, u, side="left") + lo).astype(np.int64)


def mixed(seed=SEED_BASE + 3, n_clips=200_000, sizes=(64, 128, 256), ratio=(4, 3, 1),
          jitter=4, w_lo=4, w_hi=32, zipf_s=1.2, max_list=4096, templates_per_class=None):
    """Mixed raster sizes with per-clip windows and Zipf candidate lists.

    Returns ``(clips, rep, mem)``: directed candidate pairs (member ``mem[k]``
    against representative ``rep[k]``), both of the same raster size.  Each
    clip's list holds same-template clips first, then uniform same-size clips.
    """
    rng = np.random.default_rng(seed)
    ratio = np.asarray(ratio, dtype=np.float64)
    counts = np.floor(n_clips * ratio / ratio.sum()).astype(np.int64)
    counts[0] += n_clips - counts.sum()
    sets, t_base = [], 0
    for N, cnt in zip(sizes, counts):
        n_t = templates_per_class or max(1, int(cnt) // 50)
        tpl = make_templates(rng, n_t, N, 6, 24)
        wv = rng.integers(w_lo, w_hi + 1, size=int(cnt))
        cs = make_clips(rng, tpl, N, int(cnt), jitter, wv)
        cs.template = cs.template + t_base
        t_base += n_t
        sets.append(cs)
    clips = concat(sets)
    lens = zipf_lengths(rng, clips.n, zipf_s, 1, max_list)
    reps, mems = [], []
    by_key = {}
    for i in range(clips.n):
        by_key.setdefault((int(clips.raster_n[i]), int(clips.template[i])), []).append(i)
    by_size = {N: np.flatnonzero(clips.raster_n == N) for N in sizes}
    for i in range(clips.n):
        N = int(clips.raster_n[i])
        same = [k for k in by_key[(N, int(clips.template[i]))] if k != i]
        L = int(min(lens[i], by_size[N].size - 1))
        chosen = same[:L]
        if len(chosen) < L:
            pool = by_size[N]
            taken = set(chosen) | {i}
            while len(chosen) < L:
                cand = pool[rng.integers(0, pool.size, size=2 * (L - len(chosen)) + 4)]
                for c in cand:
                    c = int(c)
                    if c not in taken:
                        taken.add(c)
                        chosen.append(c)
                        if len(chosen) == L:
                            break
        reps.append(np.full(len(chosen), i, dtype=np.int32))
        mems.append(np.asarray(chosen, dtype=np.int32))
    clips.meta.update(name="mixed", seed=seed, cos_p=97, cos_q=100, edge_tol=2)
    return clips, np.concatenate(reps), np.concatenate(mems)


def serving(seed=SEED_BASE + 5, n_library=100_000, N=128, jitter=4, w=16,
            n_requests=200, qps=50.0, median=64, sigma=1.0, max_size=10_000, return_templates=False):
    """A representative library (one clip per template) and a request trace.

    Returns ``(library, requests)`` where ``requests`` is a list of
    ``(arrival_s, ClipSet)`` with Poisson arrivals at ``qps`` and batch sizes
    ``round(LogNormal(ln median, sigma))`` clipped to [1, max_size].
    """
    rng = np.random.default_rng(seed)
    tpl = make_templates(rng, n_library, N, 6, 24)
    lib = make_clips(rng, tpl, N, n_library, jitter, w, template_of=np.arange(n_library))
    lib.meta.update(name="serving-library", seed=seed, cos_p=19, cos_q=20)
    sizes = np.clip(np.rint(rng.lognormal(np.log(median), sigma, size=n_requests)),
                    1, max_size).astype(np.int64)
    gaps = rng.exponential(1.0 / qps, size=n_requests)
    t = np.cumsum(gaps)
    reqs = []
    for k in range(n_requests):
        cs = make_clips(rng, tpl, N, int(sizes[k]), jitter, w)
        reqs.append((float(t[k]), cs))
    if return_templates:
        return lib, reqs, tpl
    return lib, reqs


def all_pairs(n):
    """All unordered pairs (i < j) of n clips as two int32 arrays."""
    i, j = np.triu_indices(n, k=1)
    return i.astype(np.int32), j.astype(np.int32)


def same_size_pairs(clips: ClipSet, rng=None, n_pairs=None):
    """Unordered pairs with equal raster size (all of them, or a uniform sample)."""
    out_i, out_j = [], []
    for N in np.unique(clips.raster_n):
        idx = np.flatnonzero(clips.raster_n == N)
        a, b = np.triu_indices(idx.size, k=1)
        out_i.append(idx[a])
        out_j.append(idx[b])
    i = np.concatenate(out_i).astype(np.int32)
    j = np.concatenate(out_j).astype(np.int32)
    if n_pairs is not None and n_pairs < i.size:
        rng = rng or np.random.default_rng(0)
        pick = np.sort(rng.choice(i.size, size=n_pairs, replace=False))
        i, j = i[pick], j[pick]
    return i, j
