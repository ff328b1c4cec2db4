"""Plant plausible mistakes in a copy of the oracle and check that the pins catch each.

Every variant is a text substitution in a temporary copy of ``nlist_oracle.c``
compiled with gcc on the CPU; the real oracle is never modified.  A variant
"survives" if every pin below still passes with it, which would mean the pins
cannot tell that mistake apart from the definition.
"""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
import workloads as W

SRC = os.path.join(os.path.dirname(oracle.__file__), "nlist_oracle.c")

MUTANTS = {
    "strict_cutoff": ("<= r2", "< r2"),
    "no_wrap_z": ("dx[d] = diff - L[d] * round(diff / L[d]);",
                  "dx[d] = (d == 2) ? diff : diff - L[d] * round(diff / L[d]);"),
    "keep_self": ("if (j == i)\n                continue;", "(void)0;"),
    "x_edge_for_all_axes": ("L[d] * round(diff / L[d])", "L[0] * round(diff / L[0])"),
    "ignore_partner_type": ("rlist2[ti * ntypes + type_of(type, j)]", "rlist2[ti * ntypes + ti]"),
    "dropped_z_term": ("(dx[0] * dx[0] + dx[1] * dx[1]) + dx[2] * dx[2]",
                       "(dx[0] * dx[0] + dx[1] * dx[1]) + dx[1] * dx[1]"),
    "floor_not_round": ("round(diff / L[d])", "floor(diff / L[d])"),
    "sign_error": ("(double)pj[d] - (double)pi[d]", "(double)pj[d] + (double)pi[d]"),
    "half_stencil": ("for (int dz = -1; dz <= 1; ++dz)", "for (int dz = 0; dz <= 1; ++dz)"),
    "narrow_cells": ("double w = rmax * (1.0 + 1e-9);", "double w = rmax * 0.75;"),
    # band-pair counting
    "band_not_relative": ("if (dev <= rel * r)", "if (dev <= rel)"),
    "band_one_sided": ("double dev = fabs(sqrt(pair_d2(pi, pj, box)) - r);",
                       "double dev = sqrt(pair_d2(pi, pj, box)) - r;"),
    "band_squared": ("double dev = fabs(sqrt(pair_d2(pi, pj, box)) - r);",
                     "double dev = fabs(pair_d2(pi, pj, box) - r2);"),
    "band_reach_unwidened": ("double e = a > b ? a : b;", "double e = r;"),
}


def _compile(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    mutated = src.replace(old, new)
    c = tmp_path / f"{name}.c"
    c.write_text(mutated)
    so = tmp_path / f"lib{name}.so"
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-std=c11",
                    str(c), "-o", str(so), "-lm"], check=True)
    return oracle.configure(ctypes.CDLL(str(so)))


def _pins_pass() -> bool:
    """A compact subset of the oracle pins; True iff all hold."""
    def rows(pos, box, rc, skin, types=None, method="brute"):
        rc = np.asarray(rc, np.float32)
        rc = rc.reshape(1, 1) if rc.ndim == 0 else rc
        rp, cols = oracle.neighbor_lists(np.asarray(pos, np.float32), np.asarray(box, np.float32),
                                         rc, skin, types=types, method=method)
        return [set(cols[rp[i]:rp[i + 1]].tolist()) for i in range(len(rp) - 1)]

    try:
        box = [10.0, 12.0, 14.0]
        for axis in range(3):
            p = np.full((2, 3), 5.0, np.float32)
            p[0, axis] = 0.125
            p[1, axis] = box[axis] - 0.125
            for method in ("brute", "cells"):
                if rows(p, box, 0.25, 0.0, method=method) != [{1}, {0}]:
                    return False
        p = np.array([[1.0, 1.0, 1.0], [1.375, 1.5, 2.5]], np.float32)
        if rows(p, [10, 10, 10], 1.625, 0.0) != [{1}, {0}]:
            return False
        if rows(p, [10, 10, 10], 1.6249, 0.0) != [set(), set()]:
            return False
        p = np.array([[1.0, 1.0, 1.0]] * 3, np.float32)
        if rows(p, [6, 6, 6], 0.5, 0.0) != [{1, 2}, {0, 2}, {0, 1}]:
            return False
        p = np.array([[1.0, 1, 1], [2.0, 1, 1], [3.25, 1, 1], [7.0, 1, 1]], np.float32)
        t = np.array([0, 0, 1, 1], np.int32)
        rc2 = np.array([[1.0, 1.5], [1.5, 1.0]], np.float32)
        if rows(p, [12, 12, 12], rc2, 0.0, types=t) != [{1}, {0, 2}, {1}, set()]:
            return False
        pos, box = W.sc_lattice(11, 1.0)
        for method in ("brute", "cells"):
            if {len(s) for s in rows(pos, box, 3.0, 0.4, method=method)} != {170}:
                return False
        cfg = W.lj_fluid(4000)
        a = oracle.neighbor_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, method="brute")
        b = oracle.neighbor_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, method="cells")
        if not (np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])):
            return False
        expect = 0.85 * (4.0 / 3.0) * math.pi * 3.4 ** 3
        if abs(np.diff(a[0]).mean() / expect - 1.0) >= 0.015:
            return False
        # band pairs: one pair 5e-6 r inside and one 5e-6 r outside the list radius
        # (both in the relative band), one 2e-5 r outside (in neither band)
        r = float(np.float32(3.0)) + float(np.float32(0.4))
        pb = []
        for k, rel in enumerate((-5e-6, 5e-6, 2e-5)):
            pb += [[5.0 + 8.0 * k, 9.0, 9.0], [5.0 + 8.0 * k, 9.0, 9.0 + r * (1.0 + rel)]]
        for method in ("brute", "cells"):
            ra, rb = oracle.band_counts(np.array(pb), np.array([30.0, 30.0, 30.0]), [[3.0]], 0.4,
                                        method=method)
            if ra.tolist() != [1, 1, 1, 1, 0, 0] or rb.tolist() != [0] * 6:
                return False
        # a band pair just outside r whose points lie two list-radius cells apart
        w = r * (1.0 + 1e-8)
        pc = np.array([[5.0, 5.0, w - 1e-7], [5.0, 5.0, w - 1e-7 + r * (1.0 + 5e-6)]])
        ra, _ = oracle.band_counts(pc, np.array([30.0, 30.0, 9.0 * w]), [[3.0]], 0.4, method="cells")
        if ra.tolist() != [1, 1]:
            return False
    except (ValueError, RuntimeError, IndexError):
        return False
    return True


def test_pins_pass_on_the_real_oracle():
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path, monkeypatch):
    old, new = MUTANTS[name]
    lib = _compile(tmp_path, name, old, new)
    monkeypatch.setattr(oracle, "_lib", lib)
    assert not _pins_pass(), f"pins did not detect planted mistake {name!r}"
