"""The seeded workload generators produce what their recipes state.

The density workload targets a union density drawn uniformly from
[0.1, 0.6] per template through rectangle sizes only; here the density of
each generated clip is measured on the oracle's rasters and compared with its
template's target.
"""
import numpy as np

import clipgen
from oracle import raster


def test_dense_workload_density_histogram():
    cs = clipgen.dense(n_clips=4000, n_templates=400)
    dens = np.array([r.mean() for r in raster.rasters(cs)])
    target = cs.meta["template_density"][cs.template]
    # the measured densities span the recipe's range ...
    p5, p50, p95 = np.percentile(dens, [5, 50, 95])
    assert 0.08 <= p5 <= 0.15 and 0.25 <= p50 <= 0.40 and 0.48 <= p95 <= 0.65, (p5, p50, p95)
    hist, _ = np.histogram(dens, bins=[0.1, 0.2, 0.3, 0.4, 0.5, 0.6])
    assert (hist >= 0.08 * dens.size).all(), hist
    # ... and follow each clip's target (overlaps and clipping at the raster
    # border pull the union a little below the independent-placement estimate)
    assert np.corrcoef(dens, target)[0, 1] > 0.9
    err = dens - target
    assert -0.06 <= err.mean() <= 0.0 and np.percentile(np.abs(err), 95) <= 0.12
    for lo in (0.1, 0.2, 0.3, 0.4, 0.5):
        m = (target >= lo) & (target < lo + 0.1)
        assert abs(dens[m].mean() - (lo + 0.05)) <= 0.07, (lo, dens[m].mean())


def test_workload_recipes_shapes():
    """Sizes, windows and list lengths of the recipes."""
    s = clipgen.small()
    assert s.n == 256 and (s.raster_n == 64).all() and (s.marker_w == 8).all()
    c = clipgen.c128(n_clips=2000, n_templates=40)
    assert (c.raster_n == 128).all() and (c.marker_w == 16).all()
    rng = np.random.default_rng(7)
    z = clipgen.zipf_lengths(rng, 200_000)
    assert z.min() >= 1 and z.max() <= 4096
    # Zipf(1.2): P(1) = 1 / H(1.2, 4096)
    k = np.arange(1, 4097, dtype=np.float64)
    p1 = 1.0 / (k ** -1.2).sum()
    assert abs((z == 1).mean() - p1) < 0.01
