"""Workload-level parity: cover relations, clusters and serving answers of
the library equal the FP64 oracle's on every benchmark workload, at full size
where the oracle can follow and scaled or stratified where it cannot.

The oracle's answers are stored in tests/golden/workload_*.npz, written by
tests/golden/make_config_golden.py from ``oracle/`` and ``clipgen`` only.
Bar: cover relations (members, shifts, counts or residuals) bit-exact, by
digest where they are large; clusters and centers bit-exact; scores within
1e-12.
"""
import importlib.util
import os
import sys

import numpy as np
import pytest

import clipgen

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def golden(name):
    return np.load(os.path.join(GOLDEN, f"workload_{name}.npz"), allow_pickle=False)


def _digest():
    spec = importlib.util.spec_from_file_location("make_config_golden", os.path.join(GOLDEN, "make_config_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.csr_digest


@pytest.fixture(scope="module")
def ctx():
    import paper_2512_13133_amd as ca
    c = ca.Context(0)
    yield c


def _csr(ctx, h, kind, thr, path="mixed"):
    return {k: v.cpu().numpy() for k, v in ctx.cover(h, kind, thr, path).items()}


def _check_clusters(got, g, key, label):
    assert got["n_clusters"] == int(g[f"{key}_n"]), f"{label}: cluster count"
    assert (got["rep_of"] == g[f"{key}_rep_of"]).all(), f"{label}: representatives"
    assert (got["center_shift"] == g[f"{key}_shift"]).all(), f"{label}: centers"


# ------------------------------------------------------------------ 256 clips of 64 x 64, all pairs


@pytest.mark.parametrize("path", ["fp64", "mixed"])
def test_small_workload_all_pairs(ctx, path):
    """The plain method on the 256-clip workload: the relation of all 32,640
    pairs (one alignment call, then the oracle's compaction of its output,
    and the library's pruned and compacted cover), and clusters for K = 1, 3."""
    from oracle import cover
    g = golden("small")
    cs = clipgen.small()
    rep, mem = clipgen.all_pairs(cs.n)
    say(f"[small] path={path} clips={cs.n} pairs={rep.size}")
    h = ctx.clips(cs, fp32=True)
    out = {k: v.cpu().numpy() for k, v in ctx.align_pairs(h, rep, mem, "cosine", (19, 20), path).items()}
    full = cover.cover_csr(cs.n, rep, mem, out["bits"], out["shift"], out["count"], out["score"])
    pruned = _csr(ctx, h, "cosine", (19, 20), path)
    for label, csr in (("all pairs", full), ("ca_cover", pruned)):
        for k in ("row_ptr", "col", "shift", "value"):
            assert (csr[k] == g[f"cos_csr_{k}"]).all(), f"cosine {label}: {k}"
        assert np.abs(csr["score"] - g["cos_csr_score"]).max() <= 1e-12
    for K in (1, 3):
        _check_clusters(ctx.cluster(h, "cosine", (19, 20), iterations=K, path=path), g, f"cos_K{K}", f"cosine K={K}")
    e = _csr(ctx, h, "edge", 2)
    for k in ("row_ptr", "col", "shift", "value"):
        assert (e[k] == g[f"edge_csr_{k}"]).all(), f"edge: {k}"
    for K in (1, 3):
        _check_clusters(ctx.cluster(h, "edge", 2, iterations=K), g, f"edge_K{K}", f"edge K={K}")
    say(f"[small] cosine nnz={g['cos_csr_col'].size} clusters K=1 {int(g['cos_K1_n'])} K=3 {int(g['cos_K3_n'])}; "
        f"edge nnz={g['edge_csr_col'].size} clusters K=1 {int(g['edge_K1_n'])} K=3 {int(g['edge_K3_n'])}")
    h.close()


@pytest.mark.parametrize("key,K,relax", [("cos_K3r1", 3, (1, 100)), ("cos_K3r4", 3, (4, 100)),
                                         ("cos_K4r3", 4, (3, 100)), ("cos_K3r0", 3, (0, 1)),
                                         ("edge_K3s2", 3, 2)])
def test_small_workload_relaxation_schedules(ctx, key, K, relax):
    """Coarse-to-fine schedules other than the default (ca_cluster_schedule)
    on the 256-clip workload: clusters and centers equal the oracle loop's."""
    g = golden("small")
    cs = clipgen.small()
    h = ctx.clips(cs, fp32=True)
    kind, thr = ("edge", 2) if key.startswith("edge") else ("cosine", (19, 20))
    got = ctx.cluster(h, kind, thr, iterations=K, relax=relax)
    _check_clusters(got, g, key, key)
    say(f"[small] {key}: {got['n_clusters']} clusters, equal to the oracle")
    h.close()


# ------------------------------------------------------------------ 128 x 128 workload at 1:10


def test_c128_workload_scaled_cosine(ctx):
    g = golden("c128s")
    digest = _digest()
    cs = clipgen.c128(n_clips=5000, n_templates=100)
    say(f"[c128/10] cosine clips={cs.n}")
    h = ctx.clips(cs, fp32=True)
    c = _csr(ctx, h, "cosine", (19, 20), "mixed")
    assert c["col"].size == int(g["cos_nnz"])
    assert digest(c["row_ptr"], c["col"], c["shift"], c["value"]) == str(g["cos_digest"])
    for K in (1, 3):
        _check_clusters(ctx.cluster(h, "cosine", (19, 20), iterations=K, path="mixed"), g, f"cos_K{K}",
                        f"cosine K={K}")
    say(f"[c128/10] nnz={c['col'].size}, oracle candidates {int(g['n_candidates'])}, clusters "
        f"K=1 {int(g['cos_K1_n'])} K=3 {int(g['cos_K3_n'])}")
    h.close()


def test_c128_workload_scaled_edge(ctx):
    g = golden("c128edge")
    digest = _digest()
    cs = clipgen.c128(n_clips=5000, n_templates=100)
    say(f"[c128/10] edge clips={cs.n}")
    h = ctx.clips(cs)
    e = _csr(ctx, h, "edge", 3)
    assert e["col"].size == int(g["edge_nnz"])
    assert digest(e["row_ptr"], e["col"], e["shift"], e["value"]) == str(g["edge_digest"])
    for K in (1, 3):
        _check_clusters(ctx.cluster(h, "edge", 3, iterations=K), g, f"edge_K{K}", f"edge K={K}")
    say(f"[c128/10] edge nnz={e['col'].size}, oracle candidates {int(g['n_candidates'])}, clusters "
        f"K=1 {int(g['edge_K1_n'])} K=3 {int(g['edge_K3_n'])}")
    h.close()


# ------------------------------------------------------------------ density workload, scaled


def test_dense_workload_scaled(ctx):
    """1:100 (20,000 clips, 200 templates) for the cosine track, 1:1000 for the
    edge track; three coarse-to-fine iterations each."""
    digest = _digest()
    g = golden("dense")
    cs = clipgen.dense(n_clips=20000, n_templates=200)
    say(f"[dense/100] cosine clips={cs.n}")
    h = ctx.clips(cs, fp32=True, fp64=False)
    c = _csr(ctx, h, "cosine", (19, 20), "mixed")
    assert c["col"].size == int(g["cos_nnz"])
    assert digest(c["row_ptr"], c["col"], c["shift"], c["value"]) == str(g["cos_digest"])
    _check_clusters(ctx.cluster(h, "cosine", (19, 20), iterations=3, path="mixed"), g, "cos_K3", "cosine K=3")
    say(f"[dense/100] nnz={c['col'].size}, oracle candidates {int(g['n_candidates'])}, "
        f"clusters K=3 {int(g['cos_K3_n'])}")
    h.close()
    ge = golden("denseedge")
    cs = clipgen.dense(n_clips=2000, n_templates=20)
    h = ctx.clips(cs)
    e = _csr(ctx, h, "edge", 2)
    assert e["col"].size == int(ge["edge_nnz"])
    assert digest(e["row_ptr"], e["col"], e["shift"], e["value"]) == str(ge["edge_digest"])
    _check_clusters(ctx.cluster(h, "edge", 2, iterations=3), ge, "edge_K3", "edge K=3")
    say(f"[dense/1000] edge nnz={e['col'].size}, clusters K=3 {int(ge['edge_K3_n'])}")
    h.close()


# ------------------------------------------------------------------ serving: 100,000-clip library


def test_serving_full_library_first_requests(ctx):
    """The serving library at full size (100,000 representatives) and the first
    request batches of the trace (>= 1,000 clips): every clip's best match,
    shift, score and cover bit equal the oracle's, with the requests in flight
    together on three slots."""
    import paper_2512_13133_amd as ca
    g = golden("serving")
    lib, reqs = clipgen.serving()
    take = [r for _, r in reqs[: int(g["n_requests"])]]
    say(f"[serving] library={lib.n} requests={len(take)} clips={sum(r.n for r in take)}")
    hlib = ctx.clips(lib, fp32=True)
    srv = ca.Server(ctx, hlib, (19, 20), slots=3)
    ids = [srv.submit(r) for r in take]
    got = []
    for rid, r in zip(ids, take):
        srv.wait(rid)
        got.append(srv.poll(rid, r.n))
    best = np.concatenate([x["best_rep"] for x in got])
    score = np.concatenate([x["score"] for x in got])
    shift = np.concatenate([x["shift"] for x in got])
    matched = np.concatenate([x["matched"] for x in got])
    assert (best == g["best"]).all()
    assert (matched == g["matched"]).all()
    ok = g["best"] >= 0
    assert (shift[ok] == g["shift"][ok]).all()
    assert np.abs(score - g["score"]).max() <= 1e-12
    rs = srv.run_stats()
    say(f"[serving] {int(ok.sum())} of {best.size} clips matched, all equal to the oracle; FP64 check of "
        f"{rs['check_pairs']} decided pairs: {rs['check_changed']} changed, peak error {rs['check_peak_err_sqrt']:.4f}")
    assert rs["check_pairs"] > 0 and rs["check_changed"] == 0
    srv.close()
    hlib.close()
