"""Surprisal-based greedy set cover, eager and lazy (paper Sec. 3.3, Eqs. 7-9).

Graph frequency f_i = 1 + |neighbours(i)| (Eq. 7), surprisal S_i = 1/f_i
(Eq. 8), and the score of a candidate representative j over the uncovered
set U, Score_j = S_j + sum_{k in neighbours(j), k in U} S_k (Eq. 9).

Readings fixed here (covers may be asymmetric when windows differ):

* "neighbours" in f_i are the nodes that can cover i (in-degree within the
  pool); in Score_j they are the nodes j covers (out-neighbours).
* Candidates are the uncovered nodes; a selected j assigns itself and every
  uncovered node it covers.
* Score_j is summed in FP64 in a fixed order: S_j first, then S_k in
  ascending k.  Ties in score go to the smaller index.
* Lazy evaluation (Sec. 3.3.2) re-computes the popped candidate's score and
  selects it when (score, -index) is at least the stale key on top of the
  heap; otherwise it is pushed back.  Stale keys are upper bounds (the fixed
  order sum of positive terms can only drop when terms are removed), so the
  lazy solver makes exactly the eager choices.
"""
from __future__ import annotations

import heapq

import numpy as np


def _adjacency(pool, covers):
    """out[j] (sorted) and in-degree f for the pool; covers is a dense bool matrix."""
    pool = np.asarray(pool, dtype=np.int64)
    sub = covers[np.ix_(pool, pool)].copy()
    np.fill_diagonal(sub, False)
    out = [np.flatnonzero(sub[a]) for a in range(pool.size)]
    f = 1 + sub.sum(axis=0)
    return out, f


def _score(j, out_j, S, uncovered):
    total = S[j]
    for k in out_j:
        if uncovered[k]:
            total = total + S[k]
    return total


def eager(pool, covers):
    """Eager greedy: returns (reps in selection order, assign dict node->rep)."""
    pool = np.asarray(pool, dtype=np.int64)
    out, f = _adjacency(pool, covers)
    S = 1.0 / f.astype(np.float64)
    uncovered = np.ones(pool.size, dtype=bool)
    reps, assign = [], {}
    while uncovered.any():
        best, best_key = -1, None
        for j in np.flatnonzero(uncovered):
            key = (_score(j, out[j], S, uncovered), -int(j))
            if best_key is None or key > best_key:
                best, best_key = int(j), key
        reps.append(int(pool[best]))
        for k in [best] + [int(k) for k in out[best] if uncovered[k]]:
            uncovered[k] = False
            assign[int(pool[k])] = int(pool[best])
    return reps, assign


def lazy(pool, covers, stats=None):
    """Lazy greedy with a max-heap of stale scores; same choices as eager()."""
    pool = np.asarray(pool, dtype=np.int64)
    out, f = _adjacency(pool, covers)
    S = 1.0 / f.astype(np.float64)
    uncovered = np.ones(pool.size, dtype=bool)
    heap = [(-_score(j, out[j], S, uncovered), j) for j in range(pool.size)]
    heapq.heapify(heap)
    reps, assign, evals = [], {}, 0
    while heap:
        neg, j = heapq.heappop(heap)
        if not uncovered[j]:
            continue
        sc = _score(j, out[j], S, uncovered)
        evals += 1
        if heap and (sc, -j) < (-heap[0][0], -heap[0][1]):
            heapq.heappush(heap, (-sc, j))
            continue
        reps.append(int(pool[j]))
        for k in [j] + [int(k) for k in out[j] if uncovered[k]]:
            uncovered[k] = False
            assign[int(pool[k])] = int(pool[j])
    if stats is not None:
        stats["evaluations"] = evals
    return reps, assign
