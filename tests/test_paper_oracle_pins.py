"""Pins of the paper-mode oracle (leaf-box overlap lists, Section 2.3): a
hand-built pair whose cell box, not its point, lies within the cutoff; the
superset relation to the exact lists; the false-positive count against the
closed form (the paper's Section 4.1 figure is reproduced from it); and
monotonicity in the pad."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import paper as P


def _pair_config(xj):
    # root box from (1,1,1) to (13.75,1,1): extent 12.75, 8 bits -> h = 12.75 / 255 = 0.05
    pos = np.array([[1.0, 1.0, 1.0], [13.75, 1.0, 1.0], [3.0, 5.0, 5.0], [xj, 5.0, 5.0]], np.float32)
    return pos, np.full(3, 20.0, np.float32)


def test_cell_box_not_point_decides():
    # x_j = 6.42: point distance 3.42 > R = 3.4, but q_lo = floor(5.42 / 0.05) = 108 puts the
    # box's lower face at 6.40, exactly R from the query: listed (eq. (2) is inclusive)
    pos, box = _pair_config(6.42)
    rp, cols = P.paper_lists(pos, box, [[3.0]], 0.4, qbits=8)
    assert 3 in cols[rp[2]:rp[3]]
    # the relation is not symmetric: i = 3 tests its point against the box of
    # particle 2, which sits on a grid line (a zero-width box 3.42 away)
    assert 2 not in cols[rp[3]:rp[4]]
    erp, ecols = oracle.neighbor_lists(pos, box, np.array([[3.0]], np.float32), 0.4)
    assert 3 not in ecols[erp[2]:erp[3]]
    # x_j = 6.46: q_lo = 109, face at 6.45, 3.45 from the query: not listed
    pos, box = _pair_config(6.46)
    rp, cols = P.paper_lists(pos, box, [[3.0]], 0.4, qbits=8)
    assert 3 not in cols[rp[2]:rp[3]]


def test_cell_boxes_contain_points_and_span_one_cell():
    cfg = W.lj_fluid(4000)
    lo, hi, h = P.cell_boxes(cfg.pos, cfg.box, None, 1, 10)
    x = cfg.pos.astype(np.float64)
    assert np.all(lo <= x) and np.all(x <= hi)
    assert np.all(hi - lo <= h * (1 + 1e-12))


@pytest.mark.parametrize("qbits", [8, 10])
def test_superset_of_exact_lists(qbits):
    cfg = W.lj_fluid(4000)
    rp, cols = P.paper_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, qbits=qbits)
    erp, ecols = oracle.neighbor_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin)
    for i in range(cfg.n):
        assert set(ecols[erp[i]:erp[i + 1]].tolist()) <= set(cols[rp[i]:rp[i + 1]].tolist())


@pytest.mark.parametrize("qbits", [8, 10])
def test_false_positives_match_the_closed_form(qbits):
    # ideal gas at the LJ density: extra entries per particle = rho (h^3 + 6 h^2 R + 3 pi h R^2)
    n, rho = 4000, 0.85
    L = (n / rho) ** (1.0 / 3.0)
    box = np.full(3, L, np.float32)
    pos, box = W.uniform(n, box, 4242)
    rcut = np.array([[3.0]], np.float32)
    rp, _ = P.paper_lists(pos, box, rcut, 0.4, qbits=qbits)
    erp, _ = oracle.neighbor_lists(pos, box, rcut, 0.4)
    fp = float((np.diff(rp) - np.diff(erp)).mean())
    _, _, h = P.cell_boxes(pos, box, None, 1, qbits)
    want = P.false_positive_mean(n / float(np.prod(box.astype(np.float64))), 3.4, h[0])
    assert abs(fp - want) <= 0.25 * want, (fp, want)


def test_bins_are_per_axis_on_a_long_box():
    # root box about 10 x 10 x 40: 8-bit bins of about 0.039, 0.039 and 0.157 sigma.
    # The false positives follow the per-axis closed form (Steiner's formula for a
    # 0.039 x 0.039 x 0.157 box) and are about half of what one 0.157 bin would give.
    n = 2000
    pos, box = W.uniform(n, [10.0, 10.0, 40.0], 4343)
    rcut = np.array([[1.6]], np.float32)
    rp, _ = P.paper_lists(pos, box, rcut, 0.4, qbits=8)
    erp, _ = oracle.neighbor_lists(pos, box, rcut, 0.4)
    fp = float((np.diff(rp) - np.diff(erp)).mean())
    _, _, h = P.cell_boxes(pos, box, None, 1, 8)
    assert h[0, 2] > 3.5 * h[0, 0] and abs(h[0, 0] - h[0, 1]) < 0.01 * h[0, 0]
    rho = n / 4000.0
    R = float(np.float32(1.6)) + float(np.float32(0.4))
    want = P.false_positive_mean(rho, R, h[0])
    iso = P.false_positive_mean(rho, R, h[0].max())
    assert abs(fp - want) <= 0.25 * want and fp < 0.7 * iso, (fp, want, iso)


def test_per_axis_bins_hand_pair():
    # root box [1, 11] x [1, 11] x [1, 41] (particles 0 and 1 at opposite corners),
    # 8 bits: h_x = 10/255 = 0.0392, h_z = 40/255 = 0.1569; R = 3.0 + 0.42.
    # Along x, particle 3 is 3.46 from particle 2 and its cell starts at
    # 1 + 139 h_x = 6.451, 3.451 away: not listed (one 0.1569 bin on every axis
    # would put the face at 6.333 and list it).  Along z, particle 5 is 3.43 from
    # particle 4 and its cell starts at 1 + 79 h_z = 13.392, 3.392 away: listed.
    pos = np.array([[1.0, 1.0, 1.0], [11.0, 11.0, 41.0], [3.0, 6.0, 20.0], [6.46, 6.0, 20.0],
                    [6.0, 3.0, 10.0], [6.0, 3.0, 13.43]], np.float32)
    box = np.array([30.0, 30.0, 60.0], np.float32)
    rp, cols = P.paper_lists(pos, box, [[3.0]], 0.42, qbits=8)
    assert 3 not in cols[rp[2]:rp[3]]
    assert 5 in cols[rp[4]:rp[5]]
    lo, hi, h = P.cell_boxes(pos, box, None, 1, 8)
    assert np.allclose(h[0], [10 / 255, 10 / 255, 40 / 255], rtol=1e-12)
    assert abs(lo[3, 0] - (1 + 139 * 10 / 255)) < 1e-12 and abs(lo[5, 2] - (1 + 79 * 40 / 255)) < 1e-12


def test_paper_figure_reproduced_by_the_closed_form():
    # Section 4.1 quotes about 1.5 extra neighbors per particle for the LJ fluid at 10 bits
    L = (4000 / 0.85) ** (1.0 / 3.0)
    want = P.false_positive_mean(0.85, 3.4, L / 1023.0)
    assert 1.3 < want < 1.7


def test_pad_is_monotone():
    cfg = W.lj_fluid(4000)
    rp0, c0 = P.paper_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, qbits=10)
    rp1, c1 = P.paper_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, qbits=10, pad=0.5)
    assert np.all(np.diff(rp1) >= np.diff(rp0))
    for i in range(0, cfg.n, 37):
        assert set(c0[rp0[i]:rp0[i + 1]].tolist()) <= set(c1[rp1[i]:rp1[i + 1]].tolist())
