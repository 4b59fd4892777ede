"""GPU parity of the cover relation (ca_cover, ca_cover_dense), the center
verification (ca_verify_centers) and clusters built on the compacted cover,
against the FP64 oracle.

Bar: row pointers, members, shifts and counts/residuals bit-exact; scores
within 1e-12 (both sides divide the same integers); clusters and centers
bit-exact; zero violations on every cluster the library returns.
"""
import sys

import numpy as np
import pytest

import clipgen
from oracle import cover

pytestmark = pytest.mark.gpu

WORKERS = 8


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import paper_2512_13133_amd as ca
    c = ca.Context(0)
    yield c


def _np(d):
    return {k: v.cpu().numpy() for k, v in d.items()}


def _check_csr(got, ref, label):
    assert (got["row_ptr"] == ref["row_ptr"]).all(), f"{label}: row pointers"
    assert (got["col"] == ref["col"]).all(), f"{label}: members"
    assert (got["shift"] == ref["shift"]).all(), f"{label}: shifts"
    assert (got["value"] == ref["value"]).all(), f"{label}: counts"
    if ref["score"].size:
        assert np.abs(got["score"] - ref["score"]).max() <= 1e-12, f"{label}: scores"


def _dense_ref(n, csr):
    words = (n + 63) // 64
    out = np.zeros((n, words), np.uint64)
    for r in range(n):
        out[r, r >> 6] |= np.uint64(1) << np.uint64(r & 63)
        for e in range(csr["row_ptr"][r], csr["row_ptr"][r + 1]):
            m = int(csr["col"][e])
            out[r, m >> 6] |= np.uint64(1) << np.uint64(m & 63)
    return out


@pytest.fixture(scope="module")
def small_case():
    cs = clipgen.small(n_clips=96)
    rep, mem = clipgen.all_pairs(cs.n)
    res = cover.align_pairs_cosine(cs, rep, mem, 19, 20, workers=WORKERS)
    er = cover.align_pairs_edge(cs, rep, mem, 2, workers=WORKERS)
    return cs, rep, mem, res, er


def test_cover_csr_and_dense_equal_oracle_small(ctx, small_case):
    cs, rep, mem, res, er = small_case
    say(f"[cover] small n={cs.n} pairs={rep.size}")
    h = ctx.clips(cs, fp32=True)
    ref_c = cover.cover_csr(cs.n, rep, mem, res["bits"], res["shift"], res["c"], res["score"])
    for path in ("fp32", "fp64", "auto"):
        _check_csr(_np(ctx.cover(h, "cosine", (19, 20), path)), ref_c, f"cosine {path}")
    dense = ctx.cover_dense(h, "cosine", (19, 20), "fp32").cpu().numpy().view(np.uint64)
    assert (dense == _dense_ref(cs.n, ref_c)).all()
    zeros = np.zeros_like(er["E"], dtype=np.float64)
    ref_e = cover.cover_csr(cs.n, rep, mem, er["bits"], er["shift"], er["E"], zeros)
    _check_csr(_np(ctx.cover(h, "edge", 2)), ref_e, "edge")
    dense = ctx.cover_dense(h, "edge", 2).cpu().numpy().view(np.uint64)
    assert (dense == _dense_ref(cs.n, ref_e)).all()
    say(f"[cover] small: cosine nnz={ref_c['col'].size} edge nnz={ref_e['col'].size}")
    h.close()


def test_cover_csr_equals_oracle_c128_mixed(ctx):
    """128 x 128 clips, window +-16, six templates: the batched mixed path with
    its FP64 re-decision feeds the compaction."""
    cs = clipgen.c128(n_clips=300, n_templates=6)
    rep, mem = clipgen.all_pairs(cs.n)
    say(f"[cover] c128 subset n={cs.n} pairs={rep.size}")
    res = cover.align_pairs_cosine(cs, rep, mem, 19, 20, workers=WORKERS)
    ref = cover.cover_csr(cs.n, rep, mem, res["bits"], res["shift"], res["c"], res["score"])
    h = ctx.clips(cs, fp32=True)
    got = _np(ctx.cover(h, "cosine", (19, 20), "mixed"))
    _check_csr(got, ref, "c128 mixed")
    lens = np.diff(ref["row_ptr"])
    say(f"[cover] c128: nnz={ref['col'].size} longest row={lens.max()}")
    assert lens.max() > 1  # rows that the one-wave sort has to order
    h.close()


def _translated_copies(n, seed):
    """n copies of one template moved by offsets in [-8, 8]^2 (rectangles kept
    inside [10, 118) so nothing is clipped): every ordered pair is an exact
    circular translation by the offset difference, within the +-16 window."""
    rng = np.random.default_rng(seed)
    base = []
    for _ in range(5):
        x0, y0 = rng.integers(10, 90, 2)
        base.append((x0, x0 + int(rng.integers(4, 28)), y0, y0 + int(rng.integers(4, 28))))
    off = rng.integers(-8, 9, size=(n, 2)).astype(np.int16)
    rects = np.array([(x0 + o[1], x1 + o[1], y0 + o[0], y1 + o[0]) for o in off for (x0, x1, y0, y1) in base],
                     np.int32)
    ptr = np.arange(0, 5 * n + 1, 5, dtype=np.int64)
    return clipgen.ClipSet(ptr, rects, np.full(n, 128, np.int16), np.full(n, 16, np.int16), np.zeros(n, np.int32),
                           off), off


@pytest.mark.parametrize("n", [300, 4400])
def test_cover_long_rows_of_translated_copies(ctx, n):
    """Closed form at any size: every clip covers every other with count n_pix,
    score 1 and shift o_m - o_r, so each row lists all other clips (rows of 299
    take the LDS sort, rows of 4,399 the chunked merge)."""
    cs, off = _translated_copies(n, seed=n)
    say(f"[cover] translated copies n={n}")
    h = ctx.clips(cs, fp32=True)
    got = _np(ctx.cover(h, "cosine", (19, 20), "mixed"))
    npix = int(ctx.inspect(h, 0, 128)["n_pix"][0])
    assert (got["row_ptr"] == np.arange(0, n * n, n - 1, dtype=np.int64)[: n + 1]).all()
    r = np.repeat(np.arange(n), n - 1)
    m = np.concatenate([np.delete(np.arange(n), i) for i in range(n)])
    assert (got["col"] == m).all()
    assert (got["shift"] == (off[m] - off[r])).all()
    assert (got["value"] == npix).all() and (got["score"] == 1.0).all()
    h.close()


@pytest.mark.parametrize("kind,thr,K", [("cosine", (19, 20), 1), ("cosine", (19, 20), 3), ("edge", 3, 3)])
def test_cluster_on_compacted_cover_c128_mixed(ctx, kind, thr, K):
    """Clusters of the mixed path equal the oracle's; every member passes the
    device center verification; planted errors are reported."""
    cs = clipgen.c128(n_clips=300, n_templates=6)
    rep, mem = clipgen.all_pairs(cs.n)
    say(f"[cluster] c128 subset {kind} K={K}")
    h = ctx.clips(cs, fp32=True)
    ctx.reset_stats()
    got = ctx.cluster(h, kind, thr, iterations=K, path="mixed")
    st = ctx.stats()
    assert st["members_verified"] == int((got["rep_of"] != np.arange(cs.n)).sum())
    assert st["center_violations"] == 0
    if kind == "cosine":
        ref = cover.cluster_cosine(cs, thr[0], thr[1], K=K, rep=rep, mem=mem, workers=WORKERS)
    else:
        ref = cover.cluster_edge(cs, thr, K=K, rep=rep, mem=mem, workers=WORKERS)
    assert got["n_clusters"] == ref["n_clusters"]
    assert (got["rep_of"] == ref["rep_of"]).all()
    assert (got["center_shift"] == ref["shift"]).all()
    assert ctx.verify_centers(h, got["rep_of"], got["center_shift"], kind, thr) == (0, -1)
    # a member moved off its center by a full window, and a representative
    # that no longer represents itself, are both caught (same as the oracle)
    members = np.flatnonzero(got["rep_of"] != np.arange(cs.n))
    if members.size:
        i = int(members[0])
        sh = got["center_shift"].copy()
        sh[i] = (17, 17)
        assert ctx.verify_centers(h, got["rep_of"], sh, kind, thr) == (1, i)
        assert cover.verify_centers(cs, got["rep_of"], sh, kind, thr) == [i]
        chain = got["rep_of"].copy()
        r = int(chain[i])
        chain[r] = i
        nv, first = ctx.verify_centers(h, chain, got["center_shift"], kind, thr)
        ref_bad = cover.verify_centers(cs, chain, got["center_shift"], kind, thr)
        assert nv == len(ref_bad) and first == ref_bad[0]
    h.close()


@pytest.mark.parametrize("kind,thr", [("cosine", (19, 20)), ("edge", 3), ("contour", 3)])
def test_prune_in_anchor_chunks_equals_one_pass(ctx, kind, thr, monkeypatch):
    """A bounds pass split into anchor chunks (a 4 KiB mask budget instead of
    the default) returns the same candidate list, in the same order, and the
    same cover relation."""
    cs = clipgen.c128(n_clips=2000, n_templates=40)
    h1 = ctx.clips(cs, contours=True)
    rep1, mem1 = (x.cpu().numpy() for x in ctx.prune(h1, kind, thr))
    cov1 = {k: v.cpu().numpy() for k, v in ctx.cover(h1, kind, thr).items()}
    h1.close()
    monkeypatch.setenv("CLIPALIGN_PRUNE_CHUNK_BYTES", "4096")
    h2 = ctx.clips(cs, contours=True)
    rep2, mem2 = (x.cpu().numpy() for x in ctx.prune(h2, kind, thr))
    cov2 = {k: v.cpu().numpy() for k, v in ctx.cover(h2, kind, thr).items()}
    h2.close()
    say(f"[prune chunks] {kind}: {rep1.size} candidates, cover entries {cov1['col'].size}")
    assert rep1.size > 0
    assert (rep1 == rep2).all() and (mem1 == mem2).all()
    for k in ("row_ptr", "col", "shift", "value"):
        assert (cov1[k] == cov2[k]).all(), k


def test_cover_in_pieces_equals_oracle_small(ctx, small_case, monkeypatch):
    """64 x 64 clips (the generic cosine bounds pass) with the candidate list
    aligned in pieces of at most n pairs: the relation still equals the
    oracle's, on both tracks."""
    cs, rep, mem, res, er = small_case
    res = cover.align_pairs_cosine(cs, rep, mem, 1, 2, workers=WORKERS)  # enough candidates at 1/2
    monkeypatch.setenv("CLIPALIGN_COVER_PIECE_PAIRS", "1")  # raised to n by the library
    h = ctx.clips(cs, fp32=True)
    n_cos = ctx.prune(h, "cosine", (1, 2))[0].numel()
    n_edge = ctx.prune(h, "edge", 2)[0].numel()
    say(f"[cover pieces] small n={cs.n}: cosine {n_cos} candidates, edge {n_edge}")
    assert n_cos > cs.n and n_edge > cs.n  # more than one piece each
    ref_c = cover.cover_csr(cs.n, rep, mem, res["bits"], res["shift"], res["c"], res["score"])
    for path in ("fp32", "auto"):
        _check_csr(_np(ctx.cover(h, "cosine", (1, 2), path)), ref_c, f"pieces cosine {path}")
    zeros = np.zeros_like(er["E"], dtype=np.float64)
    ref_e = cover.cover_csr(cs.n, rep, mem, er["bits"], er["shift"], er["E"], zeros)
    _check_csr(_np(ctx.cover(h, "edge", 2)), ref_e, "pieces edge")
    h.close()


@pytest.mark.parametrize("kind,thr", [("cosine", (19, 20)), ("edge", 3), ("contour", 3)])
def test_cover_in_pieces_equals_one_pass(ctx, kind, thr, monkeypatch):
    """128 x 128 clips (the cached bounds pass): the candidate list aligned in
    pieces of at most n pairs, with the bounds pass also in anchor chunks,
    gives the relation and the K = 3 clusters of one pass."""
    if kind == "contour":
        cs = clipgen.c128(n_clips=600, n_templates=4, jitter=1)  # equal topology within a template
    else:
        cs = clipgen.c128(n_clips=1200, n_templates=12)
    h1 = ctx.clips(cs, contours=True)
    np1 = ctx.prune(h1, kind, thr)[0].numel()
    cov1 = _np(ctx.cover(h1, kind, thr))
    cl1 = ctx.cluster(h1, kind, thr, iterations=3)
    h1.close()
    monkeypatch.setenv("CLIPALIGN_COVER_PIECE_PAIRS", "1")
    monkeypatch.setenv("CLIPALIGN_PRUNE_CHUNK_BYTES", "4096")
    h2 = ctx.clips(cs, contours=True)
    cov2 = _np(ctx.cover(h2, kind, thr))
    cl2 = ctx.cluster(h2, kind, thr, iterations=3)
    h2.close()
    say(f"[cover pieces] {kind}: n={cs.n}, {np1} candidates, cover entries {cov1['col'].size}, "
        f"clusters {cl1['n_clusters']}")
    assert np1 > cs.n and cov1["col"].size > 0
    for k in ("row_ptr", "col", "shift", "value"):
        assert (cov1[k] == cov2[k]).all(), k
    assert np.abs(cov1["score"] - cov2["score"]).max(initial=0.0) <= 1e-12
    assert cl1["n_clusters"] == cl2["n_clusters"]
    assert (cl1["rep_of"] == cl2["rep_of"]).all() and (cl1["center_shift"] == cl2["center_shift"]).all()


@pytest.mark.parametrize("path", ["xcorr", "xysep"])
def test_cover_in_pieces_other_cosine_paths(ctx, small_case, path, monkeypatch):
    """The exact objective and the XY-separation path feed the cover relation
    too: aligned in pieces of at most n pairs, the relation equals the
    one-pass relation of the same path."""
    cs = small_case[0]
    h1 = ctx.clips(cs, fp32=True)
    one = _np(ctx.cover(h1, "cosine", (1, 2), path))
    h1.close()
    monkeypatch.setenv("CLIPALIGN_COVER_PIECE_PAIRS", "1")
    h2 = ctx.clips(cs, fp32=True)
    n_cand = ctx.prune(h2, "cosine", (1, 2))[0].numel()
    pieces = _np(ctx.cover(h2, "cosine", (1, 2), path))
    h2.close()
    say(f"[cover pieces] {path}: {n_cand} candidates, {one['col'].size} entries")
    assert n_cand > cs.n and one["col"].size > 0
    for k in ("row_ptr", "col", "shift", "value"):
        assert (one[k] == pieces[k]).all(), k
    assert np.abs(one["score"] - pieces["score"]).max(initial=0.0) <= 1e-12


@pytest.mark.parametrize("kind,thr", [("cosine", (19, 20)), ("edge", 3), ("contour", 3)])
def test_prune_after_chunked_cover_equals_one_pass(ctx, kind, thr, monkeypatch):
    """The cover relation first, with the bounds pass in 4 KiB anchor chunks
    (its sizing call only plans, one sweep then counts and writes), and
    ca_prune after it (the counts are cached, each chunk's mask is rebuilt
    for the writing pass): the candidate list equals a one-pass prune's."""
    cs = clipgen.c128(n_clips=2000, n_templates=40)
    h1 = ctx.clips(cs, contours=True)
    rep1, mem1 = (x.cpu().numpy() for x in ctx.prune(h1, kind, thr))
    cov1 = _np(ctx.cover(h1, kind, thr))
    h1.close()
    monkeypatch.setenv("CLIPALIGN_PRUNE_CHUNK_BYTES", "4096")
    h2 = ctx.clips(cs, contours=True)
    cov2 = _np(ctx.cover(h2, kind, thr))
    rep2, mem2 = (x.cpu().numpy() for x in ctx.prune(h2, kind, thr))
    h2.close()
    say(f"[prune after cover] {kind}: {rep1.size} candidates, cover entries {cov1['col'].size}")
    assert rep1.size > 0
    assert (rep1 == rep2).all() and (mem1 == mem2).all()
    for k in ("row_ptr", "col", "shift", "value"):
        assert (cov1[k] == cov2[k]).all(), k
