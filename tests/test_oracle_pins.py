"""Pins for the neighbor-list oracle: values fixed by hand arithmetic, closed
forms, invariants and an independent second implementation.

Each pin is chosen so that a plausible mistake in the oracle (a dropped
periodic wrap on one axis, '<' for '<=', the self pair kept, the wrong box
edge for an axis, a type-pair lookup transposed) fails at least one of them;
``test_oracle_mutants.py`` checks exactly that by planting such mistakes.
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rows_as_sets(row_ptr, cols):
    return [set(cols[row_ptr[i]:row_ptr[i + 1]].tolist()) for i in range(len(row_ptr) - 1)]


def lists(pos, box, rc, skin, types=None, method="brute"):
    rc = np.asarray(rc, dtype=np.float32)
    if rc.ndim == 0:
        rc = rc.reshape(1, 1)
    rp, cols = oracle.neighbor_lists(np.asarray(pos, np.float32), np.asarray(box, np.float32), rc,
                                     skin, types=types, method=method)
    return rows_as_sets(rp, cols)


# ---------------------------------------------------------------- hand-built boxes

@pytest.mark.parametrize("method", ["brute", "cells"])
def test_pair_across_each_periodic_face(method):
    # distance 0.25 across the face of each axis in a box of edges 10, 12, 14
    box = [10.0, 12.0, 14.0]
    for axis in range(3):
        p = np.full((2, 3), 5.0, np.float32)
        p[0, axis] = 0.125
        p[1, axis] = box[axis] - 0.125
        assert lists(p, box, 0.25, 0.0, method=method) == [{1}, {0}]        # tie included
        assert lists(p, box, 0.2499, 0.0, method=method) == [set(), set()]  # just outside


def test_exact_tie_is_included_and_uses_rc_plus_skin():
    # (3, 4, 12) / 8 has length 13 / 8 = 1.625 exactly
    p = np.array([[1.0, 1.0, 1.0], [1.375, 1.5, 2.5]], np.float32)
    box = [10.0, 10.0, 10.0]
    assert lists(p, box, 1.225, 0.4) == [{1}, {0}]
    assert lists(p, box, 1.625, 0.0) == [{1}, {0}]
    assert lists(p, box, 1.6249, 0.0) == [set(), set()]


def test_triple_one_in_one_out_and_no_self():
    p = np.array([[2.0, 2.0, 2.0], [3.0, 2.0, 2.0], [2.0, 2.0, 4.5]], np.float32)
    got = lists(p, [8.0, 8.0, 8.0], 1.5, 0.0)
    assert got == [{1}, {0}, set()]


def test_single_and_empty():
    assert lists(np.zeros((1, 3), np.float32), [5, 5, 5], 1.0, 0.1) == [set()]
    rp, cols = oracle.neighbor_lists(np.zeros((0, 3), np.float32), [5, 5, 5], [[1.0]], 0.1)
    assert rp.tolist() == [0] and cols.size == 0


def test_coincident_particles_are_neighbors_not_self():
    p = np.array([[1.0, 1.0, 1.0]] * 3, np.float32)
    assert lists(p, [6, 6, 6], 0.5, 0.0) == [{1, 2}, {0, 2}, {0, 1}]


def test_minimum_image_not_direct_distance():
    # direct separation 9.5 but periodic separation 0.5 along y only
    p = np.array([[3.0, 0.25, 3.0], [3.0, 9.75, 3.0]], np.float32)
    assert lists(p, [7.0, 10.0, 7.0], 0.5, 0.0) == [{1}, {0}]
    assert lists(p, [7.0, 11.0, 7.0], 0.5, 0.0) == [set(), set()]


def test_type_pair_radii_and_disabled_pairs():
    # types 0,0,1,1 on a line; the 0-1 pair at distance 1.25 sits between rc[0][0] and rc[0][1]
    p = np.array([[1.0, 1, 1], [2.0, 1, 1], [3.25, 1, 1], [7.0, 1, 1]], np.float32)
    t = np.array([0, 0, 1, 1], np.int32)
    rc = np.array([[1.0, 0.0], [0.0, 4.0]], np.float32)
    assert lists(p, [12, 12, 12], rc, 0.0, types=t) == [{1}, {0}, {3}, {2}]
    rc2 = np.array([[1.0, 1.5], [1.5, 1.0]], np.float32)
    assert lists(p, [12, 12, 12], rc2, 0.0, types=t) == [{1}, {0, 2}, {1}, set()]


# ------------------------------------------------------------ closed forms

def _golden_shells():
    out = []
    with open(os.path.join(GOLDEN, "sc_shell_counts.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, c = line.split()
                out.append((int(k), int(c)))
    return out


def test_golden_shell_counts_are_lattice_sums():
    # independent check of the fixture: enumerate integer vectors directly
    for K, count in _golden_shells():
        r = int(math.isqrt(K)) + 1
        m = np.arange(-r, r + 1)
        g = m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2
        assert int(np.count_nonzero((g <= K) & (g > 0))) == count


@pytest.mark.parametrize("method", ["brute", "cells"])
def test_perfect_lattice_shell_counts(method):
    pos, box = W.sc_lattice(12, 1.0)
    for K, count in _golden_shells():
        r = math.sqrt(K + 0.5)
        rows = lists(pos, box, np.float32(r), 0.0, method=method)
        assert all(len(s) == count for s in rows), (K, count)


def test_lattice_r34_is_170_with_rc3_skin04():
    pos, box = W.sc_lattice(11, 1.0)
    rows = lists(pos, box, 3.0, 0.4, method="cells")
    assert {len(s) for s in rows} == {170}


def test_poisson_mean_count():
    # For independent uniform points in a periodic box with 2R < L, every pair is
    # within R with probability (4/3) pi R^3 / V, so E[count] = (N - 1) v / V.
    n, L, R = 20000, 30.0, 2.5
    pos, box = W.uniform(n, [L, L, L], seed=7)
    counts = oracle.neighbor_counts(pos, box, [[R]], 0.0)
    lam = (n - 1) * (4.0 / 3.0) * math.pi * R ** 3 / L ** 3
    sd = math.sqrt(2.0 * lam / n)
    assert abs(counts.mean() - lam) < 6 * sd


def test_jittered_lattice_mean_count_within_1p5_percent():
    cfg = W.lj_fluid(4000)
    counts = oracle.neighbor_counts(cfg.pos, cfg.box, cfg.rcut, cfg.skin)
    expect = 0.85 * (4.0 / 3.0) * math.pi * 3.4 ** 3
    assert abs(counts.mean() / expect - 1.0) < 0.015


# ------------------------------------------------------------ invariants

def _check_invariants(pos, box, rc, skin, types=None):
    rp, cols = oracle.neighbor_lists(pos, box, rc, skin, types=types)
    rows = rows_as_sets(rp, cols)
    for i, s in enumerate(rows):
        assert i not in s
        for j in s:
            assert i in rows[j]
    # rows are sorted ascending and duplicate-free
    for i in range(len(rows)):
        r = cols[rp[i]:rp[i + 1]]
        assert np.all(np.diff(r) > 0)
    return rp, cols


def test_symmetry_and_sorted_rows_uniform():
    pos, box = W.uniform(3000, [9.0, 11.0, 13.0], seed=3)
    _check_invariants(pos, box, [[2.0]], 0.3)


def test_symmetry_two_types():
    pos, box = W.uniform(2000, [12.0, 12.0, 12.0], seed=5)
    t = (np.arange(2000) % 3 == 0).astype(np.int32)
    rc = np.array([[1.0, 2.0], [2.0, 3.0]], np.float32)
    _check_invariants(pos, box, rc, 0.2, types=t)


# ------------------------------------------------- brute force == cell list

@pytest.mark.parametrize("maker", [
    lambda: W.lj_fluid(4000),
    lambda: W.lj_fluid(20000, seed=11),
    lambda: W.Config(*W.uniform(10000, [20.0, 24.0, 30.0], seed=9),
                     rcut=np.array([[2.2]], np.float32), skin=0.3),
])
def test_brute_equals_cells(maker):
    cfg = maker()
    a = oracle.neighbor_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, method="brute")
    b = oracle.neighbor_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, method="cells")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_brute_equals_cells_on_queries_subset():
    cfg = W.lj_fluid(20000, seed=12)
    q = np.random.default_rng(1).choice(cfg.n, 300, replace=False)
    a = oracle.neighbor_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, queries=q, method="brute")
    b = oracle.neighbor_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, queries=q, method="cells")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_generators_stay_in_half_open_box():
    for cfg in [W.lj_fluid(4000), W.lj_fluid(1000, seed=3, rho=0.3)]:
        assert cfg.pos.dtype == np.float32
        assert np.all(cfg.pos >= 0) and np.all(cfg.pos < cfg.box)
    x = np.array([[-1e-12, 10.0, 9.9999999999]])
    w = W.wrap_f32(x, np.full(3, 10.0, np.float32))
    assert np.all(w >= 0) and np.all(w < 10.0)


# ---------------------------------------------------------------- fp64 particle data

def _lists64(pos, box, rc, skin, method="brute"):
    rp, cols = oracle.neighbor_lists(np.asarray(pos, np.float64), np.asarray(box, np.float64),
                                     np.array([[rc]], np.float32), skin, method=method)
    return rows_as_sets(rp, cols)


@pytest.mark.parametrize("method", ["brute", "cells"])
def test_fp64_pairs_closer_than_fp32_resolves(method):
    # r_list = 1.5 exactly (rc 1.5 and skin 0 are exact in fp32); pairs 1.5 -/+ 1e-12
    # apart along x, at positions fp32 cannot tell apart from the tie
    r = 1.5
    box = [9.0, 9.0, 9.0]
    x0 = 3.1
    inside = np.array([[x0, 4.0, 4.0], [x0 + r - 1e-12, 4.0, 4.0]])
    outside = np.array([[x0, 4.0, 4.0], [x0 + r + 1e-12, 4.0, 4.0]])
    assert _lists64(inside, box, r, 0.0, method) == [{1}, {0}]
    assert _lists64(outside, box, r, 0.0, method) == [set(), set()]
    # the fp32 images of the two cases are the same pair of points
    assert np.array_equal(inside.astype(np.float32), outside.astype(np.float32))


def test_fp64_minimum_image_across_face():
    box = [10.0, 10.0, 10.0]
    p = np.array([[1e-13, 5.0, 5.0], [10.0 - 0.75, 5.0, 5.0]])  # 0.75 + 1e-13 apart across x
    assert _lists64(p, box, 0.75, 0.0) == [set(), set()]
    p[0, 0] = 0.0
    assert _lists64(p, box, 0.75, 0.0) == [{1}, {0}]


def test_fp64_brute_equals_cells_and_is_symmetric():
    rng = np.random.default_rng(64)
    box = np.array([13.0, 17.0, 19.0])
    pos = rng.uniform(0.0, 1.0, size=(3000, 3)) * box
    rb, cb = oracle.neighbor_lists(pos, box, np.array([[2.2]], np.float32), 0.3, method="brute")
    rc_, cc = oracle.neighbor_lists(pos, box, np.array([[2.2]], np.float32), 0.3, method="cells")
    assert np.array_equal(rb, rc_) and np.array_equal(cb, cc)
    rows = rows_as_sets(rb, cb)
    for i, s in enumerate(rows):
        assert i not in s and all(i in rows[j] for j in s)


def test_fp64_lists_differ_from_their_fp32_rounding_only_near_the_cutoff():
    # the fp64 definition is used as given: rounding the data to fp32 moves only
    # pairs whose fp64 distance is within a few fp32 ulps of r_list
    c = W.lj_fluid(4000)
    rng = np.random.default_rng(5)
    pos64 = np.mod(c.pos.astype(np.float64) + rng.uniform(-4e-7, 4e-7, size=c.pos.shape), c.box.astype(np.float64))
    box64 = c.box.astype(np.float64)
    r64, c64 = oracle.neighbor_lists(pos64, box64, c.rcut, c.skin)
    r32, c32 = oracle.neighbor_lists(pos64.astype(np.float32), c.box, c.rcut, c.skin)
    a, b = rows_as_sets(r64, c64), rows_as_sets(r32, c32)
    R = float(np.float32(c.rcut[0, 0])) + float(np.float32(c.skin))
    for i in range(c.n):
        for j in a[i] ^ b[i]:
            d = math.sqrt(oracle.pair_d2(pos64[i], pos64[j], box64))
            assert abs(d - R) < 1e-5, (i, j, d)


# ------------------------------------------------------------------ band pairs

def _r_list(rc, skin):
    return float(np.float32(rc)) + float(np.float32(skin))


@pytest.mark.parametrize("method", ["brute", "cells"])
def test_band_counts_hand_pairs(method):
    # fp64 points, so each pair sits at an exactly placed distance from r = rc + skin;
    # relative band 1e-5 * r = 3.4e-5, absolute band 1e-5
    r = _r_list(3.0, 0.4)
    box = np.array([40.0, 40.0, 40.0])
    # relative offsets of the five pairs: the first two inside the relative band,
    # the other three outside it (2e-5 r = 6.8e-5 > 3.4e-5)
    offs = [+5e-6, -5e-6, +2e-5, -2e-5, +1e-4]
    pos = []
    for k, rel in enumerate(offs):
        base = np.array([5.0 + 7.0 * k, 20.0, 20.0])
        pos += [base, base + np.array([0.0, r * (1.0 + rel), 0.0])]
    pos = np.array(pos)
    a, b = oracle.band_counts(pos, box, [[3.0]], 0.4, method=method)
    assert a.tolist() == [1, 1, 1, 1, 0, 0, 0, 0, 0, 0]
    # absolute: |d - r| = 1.7e-5 sigma for the first two pairs, above 1e-5: out
    assert b.tolist() == [0] * 10
    # a pair 0.5e-5 sigma outside r is in both bands; 2e-5 sigma outside is in the
    # relative band only (2e-5 < 3.4e-5)
    pos = np.array([[5.0, 5.0, 5.0], [5.0, 5.0, 5.0 + r + 0.5e-5],
                    [20.0, 5.0, 5.0], [20.0, 5.0, 5.0 + r + 2e-5]])
    a, b = oracle.band_counts(pos, box, [[3.0]], 0.4, method=method)
    assert a.tolist() == [1, 1, 1, 1] and b.tolist() == [1, 1, 0, 0]


def test_band_counts_reach_past_the_list_radius_cells():
    # cells exactly one list radius wide (9 along z): the pair sits 5e-6 r outside r
    # with its points two such cells apart, so the cells must be widened for the band
    r = _r_list(3.0, 0.4)
    w = r * (1.0 + 1e-8)
    pos = np.array([[5.0, 5.0, w - 1e-7], [5.0, 5.0, w - 1e-7 + r * (1.0 + 5e-6)]])
    box = np.array([30.0, 30.0, 9.0 * w])
    for method in ("brute", "cells"):
        a, _ = oracle.band_counts(pos, box, [[3.0]], 0.4, method=method)
        assert a.tolist() == [1, 1]


def test_band_counts_across_a_face_and_type_pairs():
    r = _r_list(1.0, 0.25)
    box = np.array([12.0, 12.0, 12.0])
    # a band pair across the x face, and a band pair of a disabled type pair
    pos = np.array([[0.2, 6.0, 6.0], [12.0 - (r * (1 + 2e-6) - 0.2), 6.0, 6.0],
                    [6.0, 2.0, 2.0], [6.0, 2.0, 2.0 + r]])
    types = np.array([0, 0, 1, 1], np.int32)
    rc = np.array([[1.0, 1.0], [1.0, 0.0]], np.float32)
    for method in ("brute", "cells"):
        a, b = oracle.band_counts(pos, box, rc, 0.25, types=types, method=method)
        assert a.tolist() == [1, 1, 0, 0] and b.tolist() == [1, 1, 0, 0]


def test_band_counts_brute_equals_cells_and_poisson_mean():
    # ideal gas: the expected band pairs per particle are rho * 4 pi r^2 * 2 rel r
    pos, box = W.uniform(6000, [30.0, 30.0, 30.0], seed=21)
    rel = 1e-3  # wide enough that the count is large
    a1, b1 = oracle.band_counts(pos, box, [[3.0]], 0.4, rel=rel, abs_tol=2e-3, method="brute")
    a2, b2 = oracle.band_counts(pos, box, [[3.0]], 0.4, rel=rel, abs_tol=2e-3, method="cells")
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2)
    r = _r_list(3.0, 0.4)
    rho = 6000 / 27000.0
    mean_rel = rho * 4 * math.pi * r * r * 2 * rel * r * 5999 / 6000
    mean_abs = rho * 4 * math.pi * r * r * 2 * 2e-3 * 5999 / 6000
    for got, mean in ((a1.sum(), mean_rel), (b1.sum(), mean_abs)):
        # directed pairs: each unordered pair twice, so the variance is 2 * mean * N
        sd = math.sqrt(2.0 * mean * 6000)
        assert abs(got - mean * 6000) < 6 * sd, (got, mean * 6000)
