"""Serving match rule: best covering representative per request clip (FP64).

Serving applies the refinement step of the closed loop (paper Sec. 3.1,
step 3: a pattern is aligned to fixed representatives and kept only if the
strict constraint holds, Eqs. 2-5) to clips that arrive after the library of
representatives was built.  Each request clip is aligned, as the member, to
every library clip (the fixed representative) by the cosine track of
``cosine.align``.

Reading fixed here (the paper names no rule for a clip covered by several
representatives): the best match is the covering representative with the
highest score c / sqrt(n_mem n_rep), evaluated in FP64 exactly as
``cosine.align`` reports it; equal scores go to the lowest library id.  A
clip that no representative covers gets -1, score 0 and shift (0, 0).
"""
from __future__ import annotations

import numpy as np


def best_match(n_req, req, lib, bits, score, shift):
    """Apply the rule to per-pair results.

    ``req[k]`` (request clip index), ``lib[k]`` (library clip id),
    ``bits[k]`` (True when lib[k] covers req[k]), ``score[k]`` and
    ``shift[k] = (dy, dx)`` (the request clip's displacement relative to the
    library clip) describe pair k.  Returns (best int32[n_req],
    score float64[n_req], shift int16[n_req, 2], matched uint8[n_req]).
    """
    best = np.full(n_req, -1, np.int32)
    sc = np.zeros(n_req, np.float64)
    sh = np.zeros((n_req, 2), np.int16)
    for k in range(len(req)):
        if not bits[k]:
            continue
        i, r, s = int(req[k]), int(lib[k]), float(score[k])
        if best[i] < 0 or s > sc[i] or (s == sc[i] and r < best[i]):
            best[i], sc[i], sh[i] = r, s, shift[k]
    return best, sc, sh, (best >= 0).astype(np.uint8)


def serve_match(library, request, p, q, workers=None):
    """Best match of every clip of ``request`` (a ClipSet) against every clip
    of ``library`` under the cosine constraint p/q."""
    import clipgen

    from . import cover

    both = clipgen.concat([library, request])
    nl, nr = library.n, request.n
    rep = np.repeat(np.arange(nl, dtype=np.int64), nr)
    mem = np.tile(np.arange(nl, nl + nr, dtype=np.int64), nl)
    res = cover.align_pairs_cosine(both, rep, mem, p, q, workers=workers)
    return best_match(nr, mem - nl, rep, (res["bits"] & 1).astype(bool), res["score"][:, 0], res["shift"][:, 0])
