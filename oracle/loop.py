"""Coarse-to-fine closed loop with orphan re-injection (paper Sec. 3.1).

Stage 2 clusters with relaxed thresholds via the surprisal set cover,
stage 3 accepts a member only if, aligned to its fixed representative, it
meets the strict threshold, and stage 4 re-injects the failures ("orphans")
into the next iteration until every pattern is assigned.

Readings fixed here (the paper gives no numbers for the relaxation):

* K iterations t = 1..K.  Cosine threshold tau_t = T - 0.02 (K - t)/(K - 1)
  (0.93, 0.94, 0.95 for T = 0.95, K = 3); edge threshold
  tau_t = T_edge + (K - t) px.  K = 1 uses T.  All thresholds are exact
  rationals.
* Each iteration: (1) every pool node, in ascending order, is attached to the
  first existing representative (in selection order) that covers it at the
  strict threshold; (2) the set cover runs on the remaining pool with bits at
  tau_t; (3) a member keeps its representative only if the strict bit holds,
  otherwise it stays in the pool.  The last iteration is strict, so the pool
  empties.
* Alignment runs once: the bit at any threshold is read from the stored
  overlap count (cosine) or residual (edge) of the pair's chosen shift.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

from . import scp


def cosine_schedule(p: int, q: int, K: int, relax=Fraction(2, 100)):
    """[(p_t, q_t)] for t = 1..K, exact: T - relax (K - t)/(K - 1), the total
    relaxation `relax` spread evenly over the coarse iterations."""
    T = Fraction(p, q)
    relax = Fraction(relax)
    out = []
    for t in range(1, K + 1):
        tau = T if K == 1 else T - relax * Fraction(K - t, K - 1)
        out.append((tau.numerator, tau.denominator))
    return out


def edge_schedule(t_edge: int, K: int, step: int = 1):
    """T_edge + step (K - t) pixels for t = 1..K."""
    return [t_edge + step * (K - t) for t in range(1, K + 1)]


def run(n: int, bits_at, schedule):
    """Closed loop over n nodes.

    ``bits_at(tau)`` returns a dense bool matrix covers[j, i] = "j covers i"
    at threshold tau (diagonal True).  ``schedule`` lists the K thresholds,
    the last one strict.  Returns (rep_of int64[n], reps in selection order,
    per-iteration log).
    """
    strict = bits_at(schedule[-1])
    pool = list(range(n))
    reps, rep_of, log = [], np.full(n, -1, dtype=np.int64), []
    for t, tau in enumerate(schedule):
        remaining = []
        for i in pool:
            for r in reps:
                if strict[r, i]:
                    rep_of[i] = r
                    break
            else:
                remaining.append(i)
        pool = remaining
        if not pool:
            log.append(dict(iteration=t + 1, pool=0, selected=0, orphans=0))
            continue
        sel, assign = scp.lazy(pool, bits_at(tau))
        reps += sel
        orphans = []
        for i in pool:
            r = assign[i]
            if r == i or strict[r, i]:
                rep_of[i] = r
            else:
                orphans.append(i)
        log.append(dict(iteration=t + 1, pool=len(pool), selected=len(sel), orphans=len(orphans)))
        pool = orphans
    assert not pool, "last iteration is strict, so no orphans remain"
    return rep_of, reps, log
