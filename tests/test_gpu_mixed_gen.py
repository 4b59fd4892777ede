"""GPU parity of the batched MFMA path on every raster size and window class:
64 x 64 (half-windows up to 31, and every residue for 32 and above),
128 x 128 with half-windows 17..32, and 256 x 256 up to 32, against the FP64
oracle.

Bar: shifts, overlap counts and cover bits bit-exact after the FP64
re-decision; scores within 1e-12 (both sides divide the same integers).
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


def to_np(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def check(got, ref, rep, mem, label):
    bad = np.flatnonzero((got["bits"] != ref["bits"]) | np.any(got["shift"] != ref["shift"], axis=(1, 2)) |
                         np.any(got["count"] != ref["c"], axis=1))
    if bad.size:
        k = bad[0]
        raise AssertionError(f"{label}: {bad.size} of {rep.size} pairs differ; first k={k} rep={rep[k]} mem={mem[k]} "
                             f"got shift={got['shift'][k].tolist()} c={got['count'][k].tolist()} bits={got['bits'][k]} "
                             f"ref shift={ref['shift'][k].tolist()} c={ref['c'][k].tolist()} bits={ref['bits'][k]}")
    assert np.abs(got["score"] - ref["score"]).max() <= 1e-12


def one_size_set(N, n, wmax, seed, n_templates=5):
    """n clips of raster N from a few templates (many near matches), half-windows
    drawn from {0, wmax // 2, wmax} so that pairs mix equal and unequal windows;
    the largest sets the window blocks of the launch."""
    rng = np.random.default_rng(seed)
    tpl = clipgen.make_templates(rng, n_templates, N, 3, 12)
    w = rng.choice(np.array([0, wmax // 2, wmax], np.int64), size=n)
    w[0] = wmax
    return clipgen.make_clips(rng, tpl, N, n, 4, w)


def sorted_pairs(n, n_pairs, seed):
    """Runs of equal representative (sorted), self pairs included."""
    rng = np.random.default_rng(seed)
    rep = rng.integers(0, n, n_pairs).astype(np.int32)
    mem = rng.integers(0, n, n_pairs).astype(np.int32)
    o = np.lexsort((mem, rep))
    return rep[o], mem[o]


CASES = [(64, 7), (64, 15), (64, 23), (64, 31), (64, 40),
         (128, 20), (128, 31), (128, 32),
         (256, 7), (256, 15), (256, 23), (256, 31), (256, 32)]


@pytest.mark.parametrize("N,wmax", CASES)
def test_mixed_general_kernel_equals_oracle(ctx, N, wmax):
    n = {64: 60, 128: 48, 256: 32}[N]
    cs = one_size_set(N, n, wmax, seed=N + wmax)
    rep, mem = sorted_pairs(cs.n, {64: 700, 128: 500, 256: 260}[N], seed=wmax)
    say(f"[mixed-gen] N={N} wmax={wmax} pairs={rep.size}")
    h = ctx.clips(cs, fp32=True)
    ctx.reset_stats()
    got = to_np(ctx.align_pairs(h, rep, mem, "cosine", (19, 20), "mixed"))
    st = ctx.stats()
    ref = cover.align_pairs_cosine(cs, rep, mem, 19, 20, workers=WORKERS)
    check(got, ref, rep, mem, f"N={N} w<={wmax}")
    say(f"[mixed-gen] N={N} wmax={wmax}: {int((got['bits'] != 0).sum())} covering pairs, "
        f"rescored {st['pairs_rescored']}, full FP64 {st['pairs_full_fp64']}, "
        f"peak error {st['max_peak_err_sqrt']:.4f}; FP64 check of {st['check_pairs']} decided pairs: "
        f"{st['check_changed']} changed, error {st['check_band_frac']:.3f} of the band")
    band = st["tie_band_mixed"] * max(1.0, N / 128)  # rasters above 128 take a band proportional to N
    assert st["max_peak_err_sqrt"] < band / 2
    # the decided pairs re-evaluated on the full FP64 surface (one in 256 here) kept their answers
    assert st["check_changed"] == 0
    assert st["check_band_frac"] < 0.5
    h.close()


def test_mixed_general_kernel_periodic_ties_all_residues(ctx):
    """64 x 64 periodic stripes with every residue in the window: exactly tied
    peaks (equal FP64 values and counts) in both directions, and shifts at
    -32 whose mirror is -32 again."""
    rects = []
    ptr = [0]
    for i in range(12):
        period = 8 if i % 2 == 0 else 16
        ph = i % period
        r = [(0, 64, y, y + period // 2) for y in range(ph - period, 64, period)]
        rects += r
        ptr.append(len(rects))
    n = len(ptr) - 1
    cs = clipgen.ClipSet(np.array(ptr, np.int64), np.array(rects, np.int32), np.full(n, 64, np.int16),
                         np.array([40, 32] * (n // 2), np.int16), np.zeros(n, np.int32), np.zeros((n, 2), np.int16))
    rep, mem = clipgen.all_pairs(cs.n)
    h = ctx.clips(cs, fp32=True)
    got = to_np(ctx.align_pairs(h, rep, mem, "cosine", (19, 20), "mixed"))
    ref = cover.align_pairs_cosine(cs, rep, mem, 19, 20, workers=WORKERS)
    check(got, ref, rep, mem, "periodic 64 all residues")
    assert ((got["flags"] & 3) != 0).any()  # ties went to the FP64 re-decision
    h.close()


def test_decided_pairs_checked_in_fp64_on_density_workload(ctx):
    """Clips of the density workload (union densities 0.1-0.6), every pair of
    600 clips (179,700) through the mixed path with the FP64 check at its
    largest share (one pair in 256 re-evaluated on the full FP64 surface): no
    decision changes and the peak error of the decided pairs stays below half
    the band."""
    import paper_2512_13133_amd as ca
    c = ca.Context(0, check_sample=4096)
    cs = clipgen.dense(n_clips=600, n_templates=6)
    rep, mem = clipgen.all_pairs(cs.n)
    h = c.clips(cs, fp32=True)
    got = to_np(c.align_pairs(h, rep, mem, "cosine", (19, 20), "mixed"))
    st = c.stats()
    say(f"[check] density clips: {st['check_pairs']} decided pairs checked, {st['check_changed']} changed, "
        f"peak error {st['check_peak_err_sqrt']:.4f} (band {st['tie_band_mixed']}); "
        f"{int((got['bits'] != 0).sum())} covering pairs")
    assert st["check_pairs"] >= 500 and st["check_changed"] == 0
    assert st["check_band_frac"] < 0.5
    # the checked pairs' flags are restored: a second call without the check
    # returns the same results and flags
    c2 = ca.Context(0, check_sample=-1)
    h2 = c2.clips(cs, fp32=True)
    again = to_np(c2.align_pairs(h2, rep, mem, "cosine", (19, 20), "mixed"))
    assert c2.stats()["check_pairs"] == 0
    for k in ("bits", "shift", "count", "score", "flags"):
        assert (again[k] == got[k]).all(), k
    h.close()
    h2.close()
    c.close()
    c2.close()
