"""GPU parity of the XY-separation cosine path (CA_PATH_XYSEP, paper
Sec. 3.2.1(2)) against the oracle (`oracle/xysep.py`).

Bar: shifts, overlap counts and bits bit-exact, FP64 scores within 1e-12
(both sides divide the same integers); cover relations and clusters built on
the path equal the oracle's.
"""
import sys

import numpy as np
import pytest

import clipgen
from oracle import cover, raster

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


def to_np(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def check(got, ref, rep, mem, label):
    bad = np.flatnonzero((got["bits"] != ref["bits"]) | np.any(got["shift"] != ref["shift"], axis=(1, 2)) |
                         np.any(got["count"] != ref["c"], axis=1))
    if bad.size:
        k = bad[0]
        raise AssertionError(f"{label}: {bad.size} of {rep.size} pairs differ; first k={k} rep={rep[k]} mem={mem[k]} "
                             f"got bits={got['bits'][k]} shift={got['shift'][k].tolist()} c={got['count'][k].tolist()} "
                             f"ref bits={ref['bits'][k]} shift={ref['shift'][k].tolist()} c={ref['c'][k].tolist()}")
    assert np.abs(got["score"] - ref["score"]).max() <= 1e-12


def mixed_set(seed=7, per=(24, 16, 8)):
    """Raster sizes 64/128/256, half-windows 0..32 (full-residue windows at
    64), an empty clip and a clip whose content is clipped away."""
    rng = np.random.default_rng(seed)
    sets = []
    for N, cnt in zip((64, 128, 256), per):
        tpl = clipgen.make_templates(rng, 4, N, 3, 10)
        w = rng.integers(0, 33, size=cnt)
        sets.append(clipgen.make_clips(rng, tpl, N, cnt, 4, w))
    cs = clipgen.concat(sets)
    return clipgen.concat([cs, clipgen.ClipSet(np.array([0, 0, 1], np.int64), np.array([[200, 300, 0, 5]], np.int32),
                                               np.array([64, 64], np.int16), np.array([3, 5], np.int16),
                                               np.array([-1, -1], np.int32), np.zeros((2, 2), np.int16))])


def many_polygon_set(seed=29, n=400):
    """128 x 128 clips of low-density many-rectangle templates with 1 px
    jitter: up to about 20 polygons, correspondences of more than 8."""
    rng = np.random.default_rng(seed)
    dens = rng.uniform(0.1, 0.3, size=20)
    tpl = clipgen.make_templates(rng, 20, 128, 12, 24, density=dens)
    tof = np.resize(np.arange(20), n)
    rng.shuffle(tof)
    return clipgen.make_clips(rng, tpl, 128, n, 1, 16, template_of=tof)


def template_pairs(cs, n_pairs, seed):
    """Half same-template pairs (correspondences), half uniform same-size pairs."""
    rng = np.random.default_rng(seed)
    by_tpl = {}
    for i, t in enumerate(cs.template.tolist()):
        by_tpl.setdefault((t, int(cs.raster_n[i])), []).append(i)
    reps, mems = [], []
    for i in rng.choice(cs.n, size=n_pairs // 2, replace=cs.n < n_pairs // 2).tolist():
        mates = [j for j in by_tpl[(int(cs.template[i]), int(cs.raster_n[i]))] if j != i]
        if mates:
            reps.append(i)
            mems.append(int(rng.choice(mates)))
    r2, m2 = clipgen.same_size_pairs(cs, rng, n_pairs - len(reps))
    rep = np.concatenate([np.array(reps, np.int32), r2.astype(np.int32)])
    mem = np.concatenate([np.array(mems, np.int32), m2.astype(np.int32)])
    return rep, mem


@pytest.mark.parametrize("which", ["small", "mixed", "c128", "density", "many_polygons"])
def test_xysep_matches_oracle(ctx, which):
    if which == "small":
        cs = clipgen.small(n_clips=96)
        rep, mem = clipgen.all_pairs(cs.n)
    elif which == "mixed":
        cs = mixed_set()
        rep, mem = clipgen.same_size_pairs(cs, np.random.default_rng(4), 1500)
    elif which == "c128":
        cs = clipgen.c128(n_clips=2000, n_templates=40)
        rep, mem = template_pairs(cs, 3001, seed=5)
    elif which == "density":
        cs = clipgen.dense(n_clips=2000, n_templates=200)
        rep, mem = template_pairs(cs, 2000, seed=6)
    else:
        cs = many_polygon_set()
        rep, mem = template_pairs(cs, 1600, seed=8)
    say(f"[xysep] {which}: clips={cs.n} pairs={rep.size}")
    h = ctx.clips(cs)
    got = to_np(ctx.align_pairs(h, rep, mem, "cosine", (19, 20), "xysep"))
    ref = cover.align_pairs_xysep(cs, rep, mem, 19, 20, workers=WORKERS)
    check(got, ref, rep, mem, which)
    npoly = np.array([len(raster.components(raster.clip_raster(cs, i))[1]) for i in range(cs.n)])
    big = int((np.maximum(npoly[rep], npoly[mem]) > 8).sum())
    say(f"[xysep] {which}: equal; correspondences {int(ref['matched'].sum())} of {2 * rep.size} directions, "
        f"set bits {int((ref['bits'] & 1).sum() + (ref['bits'] >> 1).sum())}, pairs with > 8 polygons {big}")
    if which == "many_polygons":
        assert big > 100 and ref["matched"][np.maximum(npoly[rep], npoly[mem]) > 8].any()
    h.close()


def test_xysep_cover_and_clusters(ctx):
    """ca_cover and ca_cluster on the XY-separation path: the relation of the
    96-clip set equals the oracle's all-pairs relation (the safe bounds hold for
    every shift of the window, so pruning drops no covering pair), and the
    clusters for K = 1 and 3 equal the oracle loop's on the oracle's results."""
    cs = clipgen.small(n_clips=96)
    rep, mem = clipgen.all_pairs(cs.n)
    ref = cover.align_pairs_xysep(cs, rep, mem, 19, 20, workers=WORKERS)
    full = cover.cover_csr(cs.n, rep, mem, ref["bits"], ref["shift"], ref["c"], ref["score"])
    h = ctx.clips(cs)
    got = {k: v.cpu().numpy() for k, v in ctx.cover(h, "cosine", (19, 20), "xysep").items()}
    for k in ("row_ptr", "col", "shift", "value"):
        assert (got[k] == full[k]).all(), k
    assert np.abs(got["score"] - full["score"]).max() <= 1e-12
    for K in (1, 3):
        want = cover.cluster_cosine(cs, 19, 20, K=K, rep=rep, mem=mem, res=ref)
        g = ctx.cluster(h, "cosine", (19, 20), iterations=K, path="xysep")
        assert g["n_clusters"] == want["n_clusters"]
        assert (g["rep_of"] == want["rep_of"]).all() and (g["center_shift"] == want["shift"]).all()
    say(f"[xysep] cover entries {full['col'].size}, clusters K=1/3 equal")
    h.close()
