"""Safe pre-screening bounds (paper Sec. 3.1 stage 1, Table 2 row 2).

The paper pre-screens pairs with cheap features before any alignment and
reports that over 99% of pairs are filtered.  These bounds are exact upper
bounds on what alignment can reach, so a pair they reject could never pass:
the cover computed with pruning equals the cover computed without.  Pruning
always uses the loosest threshold of the coarse-to-fine schedule.

B1 (area): c <= min(n), so cos <= sqrt(min n / max n).
B2 (row/column signatures): for a shift (dy, dx),
    c(s) <= U_row(dy) = sum_y min(r_rep[y], r_mem[(y + dy) mod N])
and likewise for columns, so over the member's window
    c <= min(max_dy U_row(dy), max_dx U_col(dx)).
B3 (edge): every polygon on the fewer side (both if equal) needs a partner
on the other side whose bounding box differs by at most 2 T_edge in width and
in height, since E >= |width difference| / 2 for a matched pair.
"""
from __future__ import annotations

import numpy as np

from .cosine import window_axis


def area_pass(n_a: int, n_b: int, p: int, q: int) -> bool:
    """B1: may cos exceed p/q?  (min n) q^2 > p^2 (max n)."""
    lo, hi = min(n_a, n_b), max(n_a, n_b)
    if lo == 0:
        return False
    return lo * q * q > p * p * hi


def signature_bound(a_mem, a_rep, w_mem: int) -> int:
    """B2 bound on max_{s in window} c(s), from row and column sums."""
    N = a_mem.shape[0]
    r_m, r_r = a_mem.sum(axis=1).astype(np.int64), a_rep.sum(axis=1).astype(np.int64)
    c_m, c_r = a_mem.sum(axis=0).astype(np.int64), a_rep.sum(axis=0).astype(np.int64)
    ys = np.arange(N)
    best_row = max(int(np.minimum(r_r, r_m[(ys + d) % N]).sum()) for d in window_axis(w_mem, N))
    best_col = max(int(np.minimum(c_r, c_m[(ys + d) % N]).sum()) for d in window_axis(w_mem, N))
    return min(best_row, best_col)


def signature_pass(a_mem, a_rep, w_mem: int, p: int, q: int) -> bool:
    """B2: may c(s*)/sqrt(n_m n_r) exceed p/q for some s in the window?"""
    n_m, n_r = int(a_mem.sum()), int(a_rep.sum())
    if n_m == 0 or n_r == 0:
        return False
    b = signature_bound(a_mem, a_rep, w_mem)
    return b * b * q * q > p * p * n_m * n_r


def cosine_pair_pass(a_i, a_j, w_i, w_j, p, q) -> bool:
    """Unordered pair survives if either direction may pass B1 and B2."""
    if not area_pass(int(a_i.sum()), int(a_j.sum()), p, q):
        return False
    return signature_pass(a_i, a_j, w_i, p, q) or signature_pass(a_j, a_i, w_j, p, q)


def edge_pair_pass(box_a, box_b, t_edge: int) -> bool:
    """B3 on polygon bounding boxes (arrays [P, 4] of x0, x1, y0, y1)."""
    Pa, Pb = box_a.shape[0], box_b.shape[0]
    if Pa == 0 or Pb == 0:
        return False
    wa, ha = box_a[:, 1] - box_a[:, 0], box_a[:, 3] - box_a[:, 2]
    wb, hb = box_b[:, 1] - box_b[:, 0], box_b[:, 3] - box_b[:, 2]
    ok = (np.abs(wa[:, None] - wb[None, :]) <= 2 * t_edge) & \
         (np.abs(ha[:, None] - hb[None, :]) <= 2 * t_edge)
    if Pa <= Pb and not ok.any(axis=1).all():
        return False
    if Pb <= Pa and not ok.any(axis=0).all():
        return False
    return True


# ---- the same bounds over many pairs at once (for whole clip sets) ----------


def area_pairs(npix, p: int, q: int, ids=None):
    """B1 over all unordered pairs of the clips ``ids`` (default: all): the
    pairs (i, j), i < j, with min(n) q^2 > p^2 max(n), as two int64 arrays.
    Sorting by pixel count makes each clip's admissible partners (equal or
    larger counts) one contiguous run."""
    npix = np.asarray(npix, dtype=np.int64)
    ids = np.arange(npix.size) if ids is None else np.asarray(ids, dtype=np.int64)
    order = ids[np.argsort(npix[ids], kind="stable")]
    n_sorted = npix[order]
    # partners after position a: counts n_b with n_a q^2 > p^2 n_b (n_b >= n_a)
    end = np.searchsorted(n_sorted * (p * p), n_sorted * (q * q), side="left")
    reps, mems = [], []
    for a in range(order.size):
        if n_sorted[a] == 0 or end[a] <= a + 1:
            continue
        part = order[a + 1:end[a]]
        i = np.full(part.size, order[a], dtype=np.int64)
        reps.append(np.minimum(i, part))
        mems.append(np.maximum(i, part))
    if not reps:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(reps), np.concatenate(mems)


def signature_bound_many(r_mem, c_mem, r_rep, c_rep, w_mem: int):
    """B2 bounds of many (member, representative) pairs with one half-window:
    row / column sums as arrays [P, N]; returns int64 [P] with
    min(max_dy U_row(dy), max_dx U_col(dx)) as in ``signature_bound``."""
    N = r_mem.shape[1]
    best_row = np.zeros(r_mem.shape[0], np.int64)
    best_col = np.zeros(r_mem.shape[0], np.int64)
    for d in window_axis(w_mem, N):
        best_row = np.maximum(best_row, np.minimum(r_rep, np.roll(r_mem, -int(d), axis=1)).sum(axis=1))
        best_col = np.maximum(best_col, np.minimum(c_rep, np.roll(c_mem, -int(d), axis=1)).sum(axis=1))
    return np.minimum(best_row, best_col)


def signature_pass_many(r_mem, c_mem, n_mem, r_rep, c_rep, n_rep, w_mem: int, p: int, q: int):
    """B2 test of many directed pairs: bound^2 q^2 > p^2 n_mem n_rep (bool [P])."""
    b = signature_bound_many(r_mem, c_mem, r_rep, c_rep, w_mem).astype(object)
    nm, nr = np.asarray(n_mem).astype(object), np.asarray(n_rep).astype(object)
    ok = (b * b * q * q > p * p * nm * nr) & (nm > 0) & (nr > 0)
    return ok.astype(bool)
