"""Paper-mode neighbor lists: leaf-box overlap without a distance check.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy, brute
force over all pairs, for the small inputs the tests use.

Section 2.3 lists particle j as a neighbor of i as soon as the search sphere of
i overlaps j's leaf box, and the leaf box of a quantized tree is j's position
snapped outward to the grid of its tree (Section 2.2): the root-node box split
into 2^b - 1 bins along each axis, of width h_d on axis d, and the cell box
[root_lo_d + q_lo h_d, root_lo_d + q_hi h_d] per axis, with
q_lo = floor((x_d - root_lo_d)/h_d) and q_hi = ceil((x_d - root_lo_d)/h_d)
clamped to [0, 2^b - 1] (one tree per type, each with its own root box and
bin widths, as the tree oracle defines them).
The sphere has radius R = rc[t_i][t_j] + skin, is tested under the periodic
images of the box, and the test is eq. (2): the squared distance from the
sphere's centre to the nearest point of the box is at most R^2.  The lists are
therefore supersets of the exact lists; the extra entries are the
"false positives" of Section 4.1.

``pad`` widens R by pad * max_d h_d (the widths of j's tree), which gives the
outer bracket a computed list with a small rounding pad must fall inside.
"""
from __future__ import annotations

import math

import numpy as np

from . import tree as T


def cell_boxes(pos, box, types=None, ntypes: int = 1, qbits: int = 10):
    """World-space cell box (lo [N,3], hi [N,3]) and per-axis bin widths
    h [N,3] of every particle."""
    pos = np.asarray(pos, dtype=np.float32)
    n = pos.shape[0]
    t = np.zeros(n, np.int64) if types is None else np.asarray(types, dtype=np.int64)
    lo = np.zeros((n, 3)); hi = np.zeros((n, 3)); hs = np.zeros((n, 3))
    qmax = (1 << qbits) - 1
    for ty in range(ntypes):
        sel = np.nonzero(t == ty)[0]
        if sel.size == 0:
            continue
        p = pos[sel]
        rlo = p.min(axis=0)
        rhi = p.max(axis=0)
        h = T.grid_spacing(rlo, rhi, box, qbits)
        g = (p.astype(np.float64) - rlo.astype(np.float64)[None, :]) / h[None, :]
        qlo = np.clip(np.floor(g), 0, qmax)
        qhi = np.clip(np.ceil(g), 0, qmax)
        lo[sel] = rlo.astype(np.float64)[None, :] + qlo * h[None, :]
        hi[sel] = rlo.astype(np.float64)[None, :] + qhi * h[None, :]
        hs[sel] = h[None, :]
    return lo, hi, hs


def paper_lists(pos, box, rcut, skin, types=None, qbits: int = 10, pad: float = 0.0, queries=None):
    """(row_ptr, cols) of T_i = { j != i : dist(x_i, cellbox_j) <= R_ij + pad max_d h_j,d },
    for every particle i or, with ``queries``, for those particles in that order."""
    pos = np.asarray(pos, dtype=np.float32)
    n = pos.shape[0]
    rcut = np.asarray(rcut, dtype=np.float32)
    ntypes = rcut.shape[0]
    t = np.zeros(n, np.int64) if types is None else np.asarray(types, dtype=np.int64)
    blo, bhi, hs = cell_boxes(pos, box, types, ntypes, qbits)
    hmax = hs.max(axis=1)
    L = np.asarray(box, dtype=np.float32).astype(np.float64)
    x = pos.astype(np.float64)
    rl = np.where(rcut > 0, rcut.astype(np.float64) + float(np.float32(skin)), -1.0)
    rows = []
    for i in (range(n) if queries is None else np.asarray(queries, dtype=np.int64)):
        d2 = np.zeros(n)
        for d in range(3):
            best = None
            for m in (-1.0, 0.0, 1.0):
                c = x[i, d] + m * L[d]
                e = np.maximum(np.maximum(blo[:, d] - c, c - bhi[:, d]), 0.0)
                best = e if best is None else np.minimum(best, e)
            d2 += best * best
        r = rl[t[i], t] + pad * hmax
        ok = (rl[t[i], t] > 0) & (d2 <= r * r)
        ok[i] = False
        rows.append(np.nonzero(ok)[0])
    rp = np.zeros(len(rows) + 1, np.int64)
    rp[1:] = np.cumsum([r.size for r in rows])
    cols = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    return rp, cols


def false_positive_mean(rho: float, R: float, h) -> float:
    """Expected extra entries per particle at number density rho: the volume of
    a ball of radius R grown by a box of edges (hx, hy, hz) (Steiner's formula
    hx hy hz + 2 R (hx hy + hy hz + hz hx) + pi R^2 (hx + hy + hz) + 4/3 pi R^3)
    minus the ball, times rho.  A scalar h is a cube of edge h."""
    hx, hy, hz = np.broadcast_to(np.asarray(h, dtype=np.float64), (3,))
    return float(rho * (hx * hy * hz + 2.0 * R * (hx * hy + hy * hz + hz * hx) + math.pi * R * R * (hx + hy + hz)))
