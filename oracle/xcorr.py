"""Exact-objective alignment (test infrastructure, FP64/integer, CPU only).

Paper Sec. 3.2 states the alignment objective: the shift inside the marker
region that maximises the similarity of the two clips.  Phase correlation
(Eqs. 3-5, `cosine.align`) reaches it only for pure translations; this module
evaluates the objective itself.  For a member aligned to a fixed
representative, every shift s of the member's window (the C0 rule of
`cosine.window`) gets its overlap count

    c(s) = sum_x a_rep(x) a_mem((x + s) mod N)        (an integer)

and the chosen shift is the one with the largest c(s), ties going to the
smaller |dy| + |dx|, then to the lexicographically smaller (dy, dx) (the tie
rule of `cosine.tie_key`).  Score and bit are those of Eq. 2 at that shift.
Maximising c(s) maximises the cosine c / sqrt(n_mem n_rep), since the
denominator does not depend on s.

Every value here is an integer count, so the result is exact.
"""
from __future__ import annotations

import numpy as np

from . import cosine


def overlap_surface(a_mem: np.ndarray, a_rep: np.ndarray, w_mem: int):
    """c(s) for every shift of the member's window, straight from the
    definition: returns (shifts [|W|, 2], counts [|W|])."""
    N = a_mem.shape[0]
    shifts = cosine.window(w_mem, N)
    counts = np.array([cosine.overlap(a_rep, a_mem, int(dy), int(dx)) for dy, dx in shifts], np.int64)
    return shifts, counts


def align(a_mem, a_rep, w_mem: int, p: int, q: int):
    """Member aligned to the fixed representative by the largest overlap
    count.  Returns dict(s=(dy, dx), c, score, bit).  With an empty clip the
    result is s = (0, 0), c = 0, bit = False, as on the cosine track."""
    n_mem = int(np.count_nonzero(a_mem))
    n_rep = int(np.count_nonzero(a_rep))
    if n_mem == 0 or n_rep == 0:
        return dict(s=(0, 0), c=0, score=0.0, bit=False)
    shifts, counts = overlap_surface(a_mem, a_rep, w_mem)
    best = min(range(len(counts)),
               key=lambda t: cosine.tie_key(int(counts[t]), int(shifts[t, 0]), int(shifts[t, 1])))
    dy, dx = int(shifts[best, 0]), int(shifts[best, 1])
    c = int(counts[best])
    return dict(s=(dy, dx), c=c, score=cosine.score(c, n_mem, n_rep), bit=cosine.bit(c, n_mem, n_rep, p, q))
