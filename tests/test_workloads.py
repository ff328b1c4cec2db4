"""The seeded generators: every configuration the GPU tests and the benchmark
use is a valid input (coordinates in [0, L), a unique minimum image for the
largest list radius), and the recipes hit their stated sizes and densities."""
import numpy as np
import pytest

import workloads as W


def _valid(c):
    assert c.pos.dtype == np.float32 and c.pos.shape[1] == 3
    assert np.all(c.pos >= 0) and np.all(c.pos < c.box[None, :])
    rmax = float(np.max(c.rcut)) + float(c.skin)
    assert 2.0 * rmax * (1 + 1e-9) < float(np.min(c.box)), c.name
    if c.types is not None:
        assert c.types.min() >= 0 and c.types.max() < c.ntypes


def test_served_sims_test_scale_are_valid():
    for scale in (0.01, 0.02):
        for c in W.served_sims(n_sims=24, n_slabs=6, scale=scale):
            _valid(c)


def test_served_sims_full_recipe():
    sims = W.served_sims()
    assert len(sims) == 64
    ns = np.array([c.n for c in sims])
    assert ns.min() >= 10_000 * 0.9 and ns.max() <= 2_000_000 * 1.05
    for c in sims[:16]:
        assert tuple(c.box) == (60.0, 60.0, 240.0)
    for c in sims:
        _valid(c)


def test_ensemble_recipe():
    cfgs = W.ensemble()
    ns = np.array([c.n for c in cfgs])
    assert len(cfgs) == 256 and ns.min() >= 2000 and ns.max() <= 200_000
    assert 0.9e7 < ns.sum() < 1.3e7
    for c in cfgs:
        _valid(c)
        rho = c.n / float(np.prod(c.box.astype(np.float64)))
        assert abs(rho - c.meta["rho"]) < 1e-3 * c.meta["rho"] + 1e-6


@pytest.mark.parametrize("kw", [dict(n_systems=6, n_min=800, n_max=30_000), dict(n_systems=5, n_min=1500, n_max=20_000),
                                dict(n_systems=8, n_min=2000, n_max=40_000)])
def test_small_ensembles_used_by_the_batch_tests_are_valid(kw):
    for c in W.ensemble(**kw):
        _valid(c)


def test_mixture_recipe_small():
    c = W.colloid_solvent(n_total=3000, seed=7)
    _valid(c)
    assert c.ntypes == 2 and int((c.types == 1).sum()) == 60


def test_wca_fluid_recipe():
    c = W.wca_fluid(4000)
    _valid(c)
    assert abs(float(c.rcut[0, 0]) - 2.0 ** (1.0 / 6.0)) < 1e-6
    assert np.array_equal(c.pos, W.wca_fluid(4000).pos)  # seeded


@pytest.mark.parametrize("n", [30_000, 200_000])
def test_spinodal_recipe(n):
    c = W.spinodal(n)
    _valid(c)
    assert abs(c.n - n) < 0.1 * n
    m = c.meta
    # liquid and vapor each fill about half of the box
    v_half = 0.5 * m["L"] ** 3
    assert abs(m["n_liquid"] / v_half - 0.75) < 0.08
    assert abs(m["n_vapor"] / v_half - 0.05) < 0.01
    assert np.array_equal(c.pos, W.spinodal(n).pos)  # seeded
