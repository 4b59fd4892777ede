"""Write the stored oracle answers of the workload-level parity tests
(tests/test_gpu_configs.py).

Every number here comes from the FP64 oracle (``oracle/``) on inputs of the
seeded generators (``clipgen``); nothing is read from the GPU library.  Run on
a CPU, once per change of the oracle or the generators:

    python tests/golden/make_config_golden.py [small c128s dense c128edge denseedge mixed serving]

Workloads (candidate pairs come from the oracle's own safe bounds, which
cannot drop a covering pair, so every relation below is the full one):

* small     -- 256 clips of 64 x 64 (16 templates, window +-8), all 32,640
               pairs, no pruning; cosine 19/20 and edge 2 px: the cover
               relations and the clusters for K = 1 and 3.
* c128s     -- the 128 x 128 workload at 1:10 (5,000 clips, 100 templates,
               window +-16), cosine 19/20: bounds B1 + B2 at the loosest
               threshold of K = 3 (93/100), alignment of the survivors, the
               relation at 19/20 and the clusters for K = 1 and 3.
* c128edge  -- the same clips, edge 3 px: bound B3 at 5 px (the loosest of
               K = 3), relation at 3 px, clusters for K = 1 and 3.
* dense     -- the 2M-clip density workload at 1:100 (20,000 clips, 200
               templates, densities 0.1-0.6), cosine 19/20, K = 3.
* denseedge -- the density workload at 1:1000 (2,000 clips, 20 templates),
               edge 2 px, K = 3.
* mixed     -- the 200,000-clip mixed-size workload (41.3M pairs): a stratified
               sample of 6,000 pairs (per raster size 1,000 same-template pairs
               and 1,000 uniform pairs), cosine 97/100.
* serving   -- the 100,000-clip serving library and the first request batches
               of its trace (at least 1,000 clips): best covering
               representative of every clip, cosine 19/20.
"""
from __future__ import annotations

import hashlib
from fractions import Fraction
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import clipgen  # noqa: E402
from oracle import cover, prune, raster, serve  # noqa: E402

WORKERS = max(1, len(os.sched_getaffinity(0)))


def say(*a):
    print(*a, flush=True)


def csr_digest(row_ptr, col, shift, value):
    """sha256 of a cover relation in a fixed byte layout (int64 row pointers,
    int32 members, int16 shifts, int32 counts or residuals)."""
    h = hashlib.sha256()
    for a, t in ((row_ptr, np.int64), (col, np.int32), (shift, np.int16), (value, np.int32)):
        h.update(np.ascontiguousarray(np.asarray(a, dtype=t)).tobytes())
    return h.hexdigest()


# ------------------------------------------------------------------ per-clip tables (shared by workers)

_T = {}


def _tables(cs):
    """Pixel counts and row / column sums of every clip (one size)."""
    N = int(cs.raster_n.max())
    npix = np.zeros(cs.n, np.int64)
    rows = np.zeros((cs.n, N), np.int32)
    cols = np.zeros((cs.n, N), np.int32)
    for i in range(cs.n):
        a = raster.clip_raster(cs, i)
        npix[i] = int(a.sum())
        rows[i] = a.sum(axis=1)
        cols[i] = a.sum(axis=0)
    return npix, rows, cols


def _b2_chunk(args):
    lo, hi = args
    r, m, w, p, q = _T["r"][lo:hi], _T["m"][lo:hi], _T["w"], _T["p"], _T["q"]
    rows, cols, npix = _T["rows"], _T["cols"], _T["npix"]
    fwd = prune.signature_pass_many(rows[m], cols[m], npix[m], rows[r], cols[r], npix[r], w, p, q)
    rev = prune.signature_pass_many(rows[r], cols[r], npix[r], rows[m], cols[m], npix[m], w, p, q)
    return fwd | rev


def cosine_candidates(cs, p, q, w):
    """B1 then B2 (either direction may pass) over all pairs of a one-window set."""
    npix, rows, cols = _tables(cs)
    r, m = prune.area_pairs(npix, p, q)
    say(f"  B1: {r.size} of {cs.n * (cs.n - 1) // 2} pairs")
    _T.update(r=r, m=m, w=w, p=p, q=q, rows=rows, cols=cols, npix=npix)
    step = 20000
    chunks = [(lo, min(lo + step, r.size)) for lo in range(0, r.size, step)]
    with mp.get_context("fork").Pool(WORKERS) as pool:
        keep = np.concatenate(pool.map(_b2_chunk, chunks)) if chunks else np.zeros(0, bool)
    say(f"  B2: {int(keep.sum())} survive")
    return r[keep], m[keep]


def _b3_chunk(args):
    a0, a1 = args
    boxes, t, n = _T["boxes"], _T["t"], _T["n"]
    out_r, out_m = [], []
    for i in range(a0, a1):
        for j in range(i + 1, n):
            if prune.edge_pair_pass(boxes[i], boxes[j], t):
                out_r.append(i)
                out_m.append(j)
    return np.array(out_r, np.int64), np.array(out_m, np.int64)


def edge_candidates(cs, t):
    """B3 over all pairs."""
    boxes = [raster.components(raster.clip_raster(cs, i))[1] for i in range(cs.n)]
    _T.update(boxes=boxes, t=t, n=cs.n)
    # anchors in chunks of roughly equal pair counts
    n = cs.n
    bounds, acc, start = [], 0, 0
    target = n * (n - 1) // 2 // (WORKERS * 8) + 1
    for i in range(n):
        acc += n - 1 - i
        if acc >= target:
            bounds.append((start, i + 1))
            start, acc = i + 1, 0
    if start < n:
        bounds.append((start, n))
    with mp.get_context("fork").Pool(WORKERS) as pool:
        parts = pool.map(_b3_chunk, bounds)
    r = np.concatenate([x[0] for x in parts])
    m = np.concatenate([x[1] for x in parts])
    say(f"  B3: {r.size} of {n * (n - 1) // 2} pairs")
    return r, m


def clusters_to(out, key, cl):
    out[f"{key}_rep_of"] = np.asarray(cl["rep_of"], np.int32)
    out[f"{key}_shift"] = np.asarray(cl["shift"], np.int16)
    out[f"{key}_n"] = np.int64(cl["n_clusters"])


def relation_to(out, key, n, rep, mem, res, value_key, p_or_t=None):
    if value_key == "E":
        csr = cover.cover_csr(n, rep, mem, res["bits"], res["shift"], res["E"], np.zeros_like(res["E"], np.float64))
    else:
        csr = cover.cover_csr(n, rep, mem, res["bits"], res["shift"], res["c"], res["score"])
    out[f"{key}_nnz"] = np.int64(csr["col"].size)
    out[f"{key}_digest"] = np.array(csr_digest(csr["row_ptr"], csr["col"], csr["shift"], csr["value"]))
    return csr


# ------------------------------------------------------------------ workloads


def make_small():
    cs = clipgen.small()
    rep, mem = clipgen.all_pairs(cs.n)
    out = {}
    res = cover.align_pairs_cosine(cs, rep, mem, 19, 20, workers=WORKERS)
    csr = relation_to(out, "cos", cs.n, rep, mem, res, "c")
    for k in ("row_ptr", "col", "shift", "value", "score"):
        out[f"cos_csr_{k}"] = csr[k]
    for K in (1, 3):
        clusters_to(out, f"cos_K{K}", cover.cluster_cosine(cs, 19, 20, K=K, rep=rep, mem=mem, res=res))
    er = cover.align_pairs_edge(cs, rep, mem, 2, workers=WORKERS)
    csr = relation_to(out, "edge", cs.n, rep, mem, er, "E")
    for k in ("row_ptr", "col", "shift", "value"):
        out[f"edge_csr_{k}"] = csr[k]
    for K in (1, 3):
        clusters_to(out, f"edge_K{K}", cover.cluster_edge(cs, 2, K=K, rep=rep, mem=mem, res=er))
    # other relaxation schedules (the schedule study's parity cases)
    for key, K, relax in (("cos_K3r1", 3, Fraction(1, 100)), ("cos_K3r4", 3, Fraction(4, 100)),
                          ("cos_K4r3", 4, Fraction(3, 100)), ("cos_K3r0", 3, Fraction(0))):
        clusters_to(out, key, cover.cluster_cosine(cs, 19, 20, K=K, rep=rep, mem=mem, res=res, relax=relax))
    clusters_to(out, "edge_K3s2", cover.cluster_edge(cs, 2, K=3, rep=rep, mem=mem, res=er, step=2))
    return out


def make_c128s():
    cs = clipgen.c128(n_clips=5000, n_templates=100)
    rep, mem = cosine_candidates(cs, 93, 100, 16)
    res = cover.align_pairs_cosine(cs, rep, mem, 19, 20, workers=WORKERS)
    out = {"n_candidates": np.int64(rep.size)}
    relation_to(out, "cos", cs.n, rep, mem, res, "c")
    for K in (1, 3):
        clusters_to(out, f"cos_K{K}", cover.cluster_cosine(cs, 19, 20, K=K, rep=rep, mem=mem, res=res))
    return out


def make_c128edge():
    cs = clipgen.c128(n_clips=5000, n_templates=100)
    rep, mem = edge_candidates(cs, 5)
    er = cover.align_pairs_edge(cs, rep, mem, 3, workers=WORKERS)
    out = {"n_candidates": np.int64(rep.size)}
    relation_to(out, "edge", cs.n, rep, mem, er, "E")
    for K in (1, 3):
        clusters_to(out, f"edge_K{K}", cover.cluster_edge(cs, 3, K=K, rep=rep, mem=mem, res=er))
    return out


def make_dense():
    cs = clipgen.dense(n_clips=20000, n_templates=200)
    rep, mem = cosine_candidates(cs, 93, 100, 16)
    res = cover.align_pairs_cosine(cs, rep, mem, 19, 20, workers=WORKERS)
    out = {"n_candidates": np.int64(rep.size)}
    relation_to(out, "cos", cs.n, rep, mem, res, "c")
    clusters_to(out, "cos_K3", cover.cluster_cosine(cs, 19, 20, K=3, rep=rep, mem=mem, res=res))
    return out


def make_denseedge():
    cs = clipgen.dense(n_clips=2000, n_templates=20)
    rep, mem = edge_candidates(cs, 4)
    er = cover.align_pairs_edge(cs, rep, mem, 2, workers=WORKERS)
    out = {"n_candidates": np.int64(rep.size)}
    relation_to(out, "edge", cs.n, rep, mem, er, "E")
    clusters_to(out, "edge_K3", cover.cluster_edge(cs, 2, K=3, rep=rep, mem=mem, res=er))
    return out


def make_mixed():
    cs, rep, mem = clipgen.mixed()
    rng = np.random.default_rng(2024)
    same = cs.template[rep] == cs.template[mem]
    pick = []
    for N in (64, 128, 256):
        size = cs.raster_n[rep] == N
        pick.append(rng.choice(np.flatnonzero(size & same), 1000, replace=False))
        pick.append(rng.choice(np.flatnonzero(size), 1000, replace=False))
    pick = np.concatenate(pick)
    ids, inv = np.unique(np.concatenate([rep[pick], mem[pick]]), return_inverse=True)
    sub = cs.subset(ids)
    res = cover.align_pairs_cosine(sub, inv[:pick.size], inv[pick.size:], 97, 100, workers=WORKERS)
    say(f"  sample: {pick.size} pairs, {int((res['bits'] != 0).sum())} with a set bit")
    return {"pick": pick.astype(np.int64), "bits": res["bits"], "shift": res["shift"], "c": res["c"],
            "score": res["score"]}


def _serve_chunk(args):
    lo, hi = args
    lib_n, lib_rows, lib_cols, lib = _T["lib_n"], _T["lib_rows"], _T["lib_cols"], _T["lib"]
    req = _T["req"]
    out = []
    for i in range(lo, hi):
        a = raster.clip_raster(req, i)
        n_i = int(a.sum())
        r_i, c_i = a.sum(axis=1).astype(np.int32), a.sum(axis=0).astype(np.int32)
        cand = np.flatnonzero((np.minimum(lib_n, n_i) * 400 > 361 * np.maximum(lib_n, n_i)) & (lib_n > 0)) \
            if n_i > 0 else np.zeros(0, np.int64)
        if cand.size:
            P = cand.size
            ok = prune.signature_pass_many(np.repeat(r_i[None], P, 0), np.repeat(c_i[None], P, 0), np.full(P, n_i),
                                           lib_rows[cand], lib_cols[cand], lib_n[cand], int(req.marker_w[i]), 19, 20)
            cand = cand[ok]
        if cand.size == 0:
            out.append((-1, 0.0, 0, 0, 0, 0))
            continue
        one = req.subset([i])
        best, sc, sh, matched = serve.serve_match(lib.subset(cand), one, 19, 20)
        b = int(best[0])
        out.append((int(cand[b]) if b >= 0 else -1, float(sc[0]), int(sh[0, 0]), int(sh[0, 1]), int(matched[0]),
                    int(cand.size)))
    return out


def make_serving():
    lib, reqs = clipgen.serving()
    take, total = [], 0
    for _, r in reqs:
        take.append(r)
        total += r.n
        if total >= 1000:
            break
    req = clipgen.concat(take)
    say(f"  library {lib.n} clips, {len(take)} requests, {req.n} clips")
    lib_n, lib_rows, lib_cols = _tables(lib)
    _T.update(lib=lib, lib_n=lib_n, lib_rows=lib_rows, lib_cols=lib_cols, req=req)
    step = 16
    chunks = [(lo, min(lo + step, req.n)) for lo in range(0, req.n, step)]
    with mp.get_context("fork").Pool(WORKERS) as pool:
        rows = [x for part in pool.map(_serve_chunk, chunks) for x in part]
    rows = np.array(rows, dtype=np.float64)
    say(f"  matched {int(rows[:, 4].sum())} of {req.n}; candidates per clip: median {np.median(rows[:, 5]):.0f}")
    return {"n_requests": np.int64(len(take)), "best": rows[:, 0].astype(np.int32), "score": rows[:, 1],
            "shift": rows[:, 2:4].astype(np.int16), "matched": rows[:, 4].astype(np.uint8)}


MAKERS = {"small": make_small, "c128s": make_c128s, "c128edge": make_c128edge, "dense": make_dense,
          "denseedge": make_denseedge, "mixed": make_mixed, "serving": make_serving}


def main(argv):
    names = argv or list(MAKERS)
    for name in names:
        t = time.time()
        say(f"[golden] {name}")
        out = MAKERS[name]()
        path = os.path.join(HERE, f"workload_{name}.npz")
        np.savez_compressed(path, **out)
        say(f"[golden] {name}: {path} ({os.path.getsize(path) / 1024:.0f} KB) in {time.time() - t:.0f} s")


if __name__ == "__main__":
    main(sys.argv[1:])
