"""Pins for the step-by-step tree oracle (``oracle/tree.py``).

Each step is checked against something other than itself: hand values and the
Z-order comparison for Morton codes, Python's stable sort, a bit-by-bit
compressed trie for the radix tree, containment/union properties for the
boxes, exact rational arithmetic for the quantization, and -- for the final
node layout -- a plain CPU run of the paper's stackless traversal (Algorithm 1)
over the emitted nodes, which must reproduce the brute-force neighbor lists.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import tree as T

import layout_ref as LR


# ------------------------------------------------------------------- Morton codes

def test_morton_hand_values():
    box = np.full(3, 1023.0, np.float32)  # bin = floor(x), x in the lowest code bit
    pts = np.array([[1.5, 0.5, 0.5], [0.5, 1.5, 0.5], [0.5, 0.5, 1.5], [0.5, 0.5, 0.5],
                    [1022.5, 1022.5, 1022.5], [3.5, 0.5, 0.5]], np.float32)
    codes = T.morton_keys(pts, box)
    assert codes.tolist() == [1, 2, 4, 0, (1 << 30) - 1 - 7, 1 | 8]
    typed = T.morton_keys(pts[:2], box, types=np.array([1, 3], np.int32))
    assert typed.tolist() == [(1 << 30) | 1, (3 << 30) | 2]


def _zorder_less(a, b):
    # Z-order comparison without interleaving: the axis holding the most
    # significant differing bit decides (z outranks y outranks x on equal bits).
    best, axis = -1, 0
    for d in range(3):
        x = int(a[d]) ^ int(b[d])
        if x and x.bit_length() - 1 >= best:
            best, axis = x.bit_length() - 1, d
    return best >= 0 and int(a[axis]) < int(b[axis])


def test_morton_order_is_z_order():
    rng = np.random.default_rng(0)
    box = np.full(3, 1023.0, np.float32)
    bins = rng.integers(0, 1023, size=(400, 3))
    pts = (bins + 0.5).astype(np.float32)
    codes = T.morton_keys(pts, box)
    for _ in range(3000):
        i, j = rng.integers(0, 400, 2)
        assert (codes[i] < codes[j]) == _zorder_less(bins[i], bins[j])


def test_morton_bins_cover_the_box():
    pos, box = W.uniform(5000, [7.0, 9.0, 11.0], seed=1)
    b = np.floor(pos.astype(np.float64) * (1023.0 / box.astype(np.float64)))
    assert b.min() >= 0 and b.max() <= 1022


# ------------------------------------------------------------------------ sort

def test_sort_is_stable():
    rng = np.random.default_rng(2)
    keys = rng.integers(0, 20, size=500).astype(np.uint32)
    sk, perm = T.sort_keys(keys)
    ref = sorted(range(500), key=lambda i: (int(keys[i]), i))
    assert perm.tolist() == ref
    assert np.all(np.diff(sk.astype(np.int64)) >= 0)


# ------------------------------------------------------------------ radix tree

def _trie_nodes(sorted_keys, s, e):
    """Binary radix tree as a compressed binary trie, built bit by bit from the top."""
    a = [(int(sorted_keys[k]) << 32) | k for k in range(s, e)]
    out = {}
    stack = [(s, e - 1, 63)]
    while stack:
        f, l, bit = stack.pop()
        if f == l:
            continue
        while True:  # skip bits on which the whole range agrees (unary trie nodes)
            ones = [k for k in range(f, l + 1) if (a[k - s] >> bit) & 1]
            if 0 < len(ones) < l - f + 1:
                break
            bit -= 1
        gamma = ones[0] - 1
        out[(f, l)] = gamma
        stack.append((f, gamma, bit - 1))
        stack.append((gamma + 1, l, bit - 1))
    return out


@pytest.mark.parametrize("n,ncode", [(2, 8), (3, 2), (17, 5), (64, 1), (200, 40), (300, 1 << 30)])
def test_radix_tree_equals_compressed_trie(n, ncode):
    rng = np.random.default_rng(n)
    keys = np.sort(rng.integers(0, ncode, size=n).astype(np.uint32))
    nodes = T.radix_tree(keys, 0, n)
    assert nodes == _trie_nodes(keys, 0, n)
    # N - 1 internal nodes, two children each, every leaf below exactly one parent
    assert len(nodes) == n - 1
    child_ranges = []
    for (f, l), g in nodes.items():
        assert f <= g < l
        child_ranges += [(f, g), (g + 1, l)]
    leaves = [r for r in child_ranges if r[0] == r[1]]
    assert sorted(r[0] for r in leaves) == list(range(n))
    assert (0, n - 1) in nodes


def test_radix_tree_on_segment_offset():
    keys = np.array([5, 1 << 30, (1 << 30) + 3, (1 << 30) + 3, (1 << 30) + 9], np.uint32)
    nodes = T.radix_tree(keys, 1, 5)
    assert nodes == _trie_nodes(keys, 1, 5)
    assert (1, 4) in nodes and len(nodes) == 3


# ---------------------------------------------------------------------- boxes

def test_boxes_union_and_root():
    cfg = W.lj_fluid(1500, seed=4)
    b = T.build_steps(cfg.pos, cfg.box)
    (tree,), (boxes,) = b["trees"], b["boxes"]
    p = b["sorted_pos"]

    def box_of(f, l):
        return (p[f], p[f]) if f == l else boxes[(f, l)]

    for (f, l), g in tree.items():
        lo, hi = boxes[(f, l)]
        llo, lhi = box_of(f, g)
        rlo, rhi = box_of(g + 1, l)
        assert np.array_equal(lo, np.minimum(llo, rlo)) and np.array_equal(hi, np.maximum(lhi, rhi))
    lo, hi = boxes[(0, cfg.n - 1)]
    assert np.array_equal(lo, cfg.pos.min(axis=0)) and np.array_equal(hi, cfg.pos.max(axis=0))


# ---------------------------------------------------------------- quantization

@pytest.mark.parametrize("qbits", [10, 16])
def test_quantized_bounds_are_outward_and_within_one_bin(qbits):
    # a root box with unequal edges, so each axis has its own bin width
    pos, box = W.uniform(800, [9.0, 14.0, 23.0], seed=6)
    b = T.build_steps(pos, box)
    (boxes,) = b["boxes"]
    rlo, rhi = boxes[(0, 799)]
    h = T.grid_spacing(rlo, rhi, box, qbits)
    ext = rhi.astype(np.float64) - rlo.astype(np.float64)
    assert np.all(h * ((1 << qbits) - 1) >= ext) and h[0] < h[1] < h[2]
    tol = Fraction(1, 10 ** 9)  # fp64 evaluation error, far below the traversal's 2-bin pad
    for (f, l), (lo, hi) in list(boxes.items())[:300]:
        qlo, qhi = T.quantize_box(lo, hi, rlo, h, qbits)
        for d in range(3):
            H = Fraction(float(h[d]))
            assert 0 <= qlo[d] <= qhi[d] <= (1 << qbits) - 1
            glo = (Fraction(float(lo[d])) - Fraction(float(rlo[d]))) / H
            ghi = (Fraction(float(hi[d])) - Fraction(float(rlo[d]))) / H
            assert qlo[d] <= glo + tol and qhi[d] >= ghi - tol      # outward
            assert qlo[d] > glo - 1 and qhi[d] < ghi + 1              # at most one bin loose


def test_per_axis_bins_hand_values():
    # root box [0,2] x [0,4] x [0,8] with 2-bit bounds: 3 bins per axis of
    # widths 2/3, 4/3 and 8/3; the point (1,1,1) lies in bins 1, 0 and 0
    lo = np.zeros(3, np.float32)
    hi = np.array([2.0, 4.0, 8.0], np.float32)
    h = T.grid_spacing(lo, hi, np.full(3, 10.0, np.float32), 2)
    assert np.allclose(h, [2 / 3, 4 / 3, 8 / 3], rtol=0, atol=1e-15)
    p = np.ones(3, np.float32)
    assert T.quantize_box(p, p, lo, h, 2) == ([1, 0, 0], [2, 1, 1])
    assert T.quantize_box(lo, hi, lo, h, 2) == ([0, 0, 0], [3, 3, 3])  # the root box spans every bin


def test_grid_spacing_floor_for_coincident_points():
    lo = hi = np.array([1.0, 2.0, 3.0], np.float32)
    h = T.grid_spacing(lo, hi, np.full(3, 10.0, np.float32), 16)
    assert np.all(h == 10.0 * 2.0 ** -24 / 65535)
    # only the axis without extent is floored
    h = T.grid_spacing(lo, np.array([1.0, 5.0, 3.0], np.float32), np.full(3, 10.0, np.float32), 16)
    assert h[1] == 3.0 / 65535 and h[0] == h[2] == 10.0 * 2.0 ** -24 / 65535


def test_layout_grid_is_the_largest_axis_width():
    # the library's isotropic grid (layout helper) takes the largest per-axis width
    lo = np.zeros(3, np.float32)
    hi = np.array([2.0, 7.0, 3.0], np.float32)
    assert LR.iso_spacing(lo, hi, np.full(3, 10.0, np.float32), 10) == 7.0 / 1023


# --------------------------------------------------- layout: Algorithm 1 on the CPU

def _run(ref):
    """Decode a particle-run reference: (first, count)."""
    ref = int(ref)
    v = ~(ref - (1 << 32) if ref >= (1 << 31) else ref)
    return v >> 4, (v & 15) + 1


def _alg1_rows(records, ropes, meta, box, rlist2, qtypes, qpos, orig_of_query, sorted_pos, perm,
               types_sorted):
    """The paper's stackless traversal over the emitted records, in plain Python.

    At a record both child boxes are decoded (root lo + q * h) and tested
    against the search sphere with the nearest-point rule (eq. 2, tiny pad).
    Every particle of a hit particle run is a candidate, decided by the exact
    fp64 minimum-image distance of the list definition.  The walk goes to the
    left child's record if that box is hit, else to the right child's record
    if that box is hit, else along the rope.
    """
    L = np.asarray(box, np.float64)
    rows = []
    for qi in range(qpos.shape[0]):
        x = qpos[qi].astype(np.float64)
        ta = qtypes[qi]
        found = []
        for tb, m in enumerate(meta):
            r2 = rlist2[ta, tb]
            if m["count"] == 0 or r2 < 0:
                continue
            R = np.sqrt(r2)
            rlo = m["lo"].astype(np.float64)
            rhi = m["hi"].astype(np.float64)
            for img in range(27):
                shift = np.array([img % 3 - 1, (img // 3) % 3 - 1, img // 9 - 1], np.float64)
                c = x + shift * L
                y = np.minimum(np.maximum(c, rlo), rhi)
                if np.sum((y - c) ** 2) > r2 * (1 + 1e-12):
                    continue

                def take(first, count):
                    for k in range(first, first + count):
                        assert types_sorted[k] == tb
                        dx = (sorted_pos[k].astype(np.float64) - x) - shift * L
                        d2 = (dx[0] * dx[0] + dx[1] * dx[1]) + dx[2] * dx[2]
                        j = int(perm[k])
                        if d2 <= r2 and j != orig_of_query[qi]:
                            found.append(j)

                if m["root"] < 0:
                    take(*_run(m["root"]))
                    continue
                v = m["root"]
                while v < m["end"]:
                    w = records[v]
                    hit = []
                    for side in range(2):
                        q = w[3 * side:3 * side + 3]
                        lo = rlo + np.array([int(a) & 0xFFFF for a in q], np.float64) * m["h"]
                        hi = rlo + np.array([int(a) >> 16 for a in q], np.float64) * m["h"]
                        y = np.minimum(np.maximum(c, lo), hi)
                        hit.append(np.sqrt(np.sum((y - c) ** 2)) <= R * (1 + 1e-9) + 1e-9)
                        ref = int(np.int32(np.uint32(w[6 + side])))
                        if hit[side] and ref < 0:
                            take(*_run(ref))
                    left, right = int(np.int32(np.uint32(w[6]))), int(np.int32(np.uint32(w[7])))
                    if hit[0] and left >= 0:
                        v = left
                    elif hit[1] and right >= 0:
                        v = right
                    else:
                        v = int(ropes[v])
        rows.append(sorted(found))
    return rows


@pytest.mark.parametrize("leaf_size,qbits", [(1, 16), (1, 10), (3, 16), (8, 12), (16, 16), (13, 10)])
def test_layout_traversal_reproduces_brute_force(leaf_size, qbits):
    cfg = W.lj_fluid(350, seed=8, rho=0.6, rc=2.0, skin=0.3)
    b = LR.build_all(cfg.pos, cfg.box, leaf_size=leaf_size, qbits=qbits)
    r2 = oracle.rlist2_table(cfg.rcut, cfg.skin)
    perm = b["perm"].astype(np.int64)
    rows = _alg1_rows(b["records"], b["ropes"], b["meta"], cfg.box, r2, np.zeros(cfg.n, np.int64),
                      b["sorted_pos"], perm, b["sorted_pos"], perm, np.zeros(cfg.n, np.int64))
    rp, cols = oracle.neighbor_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, method="brute")
    for k in range(cfg.n):
        i = perm[k]
        assert rows[k] == cols[rp[i]:rp[i + 1]].tolist()
    # one record per internal node whose particle range is larger than a leaf run
    kept = sum(1 for (f, l) in b["trees"][0] if l - f + 1 > leaf_size)
    assert b["records"].shape[0] == kept


@pytest.mark.parametrize("leaf_size,radius", [(16, 2.3), (16, 0.5), (6, 1.0)])
def test_cost_collapse_layout_traversal_reproduces_brute_force(leaf_size, radius):
    cfg = W.lj_fluid(350, seed=8, rho=0.6, rc=2.0, skin=0.3)
    b = LR.build_all(cfg.pos, cfg.box, leaf_size=leaf_size, collapse_radius=radius)
    r2 = oracle.rlist2_table(cfg.rcut, cfg.skin)
    perm = b["perm"].astype(np.int64)
    rows = _alg1_rows(b["records"], b["ropes"], b["meta"], cfg.box, r2, np.zeros(cfg.n, np.int64),
                      b["sorted_pos"], perm, b["sorted_pos"], perm, np.zeros(cfg.n, np.int64))
    rp, cols = oracle.neighbor_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, method="brute")
    for k in range(cfg.n):
        assert rows[k] == cols[rp[perm[k]]:rp[perm[k] + 1]].tolist()
    # runs are whole collapsed subtrees of at most leaf_size particles covering every particle once
    left, right = b["records"][:, 6].view(np.int32), b["records"][:, 7].view(np.int32)
    covered = np.zeros(cfg.n, np.int64)
    for ref in np.concatenate([left[left < 0], right[right < 0]]):
        f, c = _run(ref)
        assert 1 <= c <= leaf_size and (c == 1 or (f, f + c - 1) in b["trees"][0])
        covered[f:f + c] += 1
    assert np.all(covered == 1)


def test_cost_collapse_reduces_to_the_size_rule_for_large_radii():
    # with spheres far larger than any node, every box grows to about the same
    # volume V: a subtree of c particles then costs c V as a run and at least
    # (4 + c) V split, so every subtree of at most leaf_size particles collapses
    cfg = W.lj_fluid(800, seed=11)
    for leaf_size in (2, 8, 16):
        a = LR.build_all(cfg.pos, cfg.box, leaf_size=leaf_size)
        b = LR.build_all(cfg.pos, cfg.box, leaf_size=leaf_size, collapse_radius=1e6)
        assert np.array_equal(a["records"], b["records"]) and np.array_equal(a["ropes"], b["ropes"])


def test_cost_collapse_keeps_spread_subtrees_split():
    # two tight clusters of 4 far apart inside one subtree of 8: split (two runs of 4)
    # beats one run of 8 for small spheres, one run of 8 wins for large ones
    pts = np.array([[1, 1, 1], [1.01, 1, 1], [1, 1.01, 1], [1.01, 1.01, 1],
                    [5, 5, 5], [5.01, 5, 5], [5, 5.01, 5], [5.01, 5.01, 5]], np.float32)
    box = np.full(3, 8.0, np.float32)
    small = LR.build_all(pts, box, leaf_size=8, collapse_radius=0.1)
    large = LR.build_all(pts, box, leaf_size=8, collapse_radius=50.0)
    assert small["records"].shape[0] == 1 and large["records"].shape[0] == 0
    runs = sorted(_run(int(np.int32(np.uint32(w)))) for w in small["records"][0, 6:8])
    assert runs == [(0, 4), (4, 4)]


def test_layout_two_types_and_empty_type():
    pos, box = W.uniform(300, [9.0, 9.0, 9.0], seed=13)
    types = (np.arange(300) % 4 == 0).astype(np.int32) * 2  # types 0 and 2, type 1 empty
    rcut = np.array([[1.2, 0.0, 1.6], [0.0, 1.0, 0.0], [1.6, 0.0, 2.0]], np.float32)
    b = LR.build_all(pos, box, types=types, ntypes=3, leaf_size=2)
    assert b["meta"][1]["count"] == 0
    r2 = oracle.rlist2_table(rcut, 0.25)
    perm = b["perm"].astype(np.int64)
    rows = _alg1_rows(b["records"], b["ropes"], b["meta"], box, r2, types[perm], b["sorted_pos"], perm,
                      b["sorted_pos"], perm, types[perm])
    rp, cols = oracle.neighbor_lists(pos, box, rcut, 0.25, types=types, method="brute")
    for k in range(300):
        i = perm[k]
        assert sorted(rows[k]) == cols[rp[i]:rp[i + 1]].tolist()


def test_layout_tree_smaller_than_a_leaf_run():
    pos = np.array([[1.0, 1.0, 1.0], [1.5, 1.0, 1.0], [6.0, 6.0, 6.0]], np.float32)
    b = LR.build_all(pos, np.full(3, 9.0, np.float32), leaf_size=4)
    (m,) = b["meta"]
    assert b["records"].shape[0] == 0 and _run(m["root"]) == (0, 3)


def test_layout_ropes_and_children():
    cfg = W.lj_fluid(500, seed=9)
    for leaf_size in (1, 2, 5, 16):
        b = LR.build_all(cfg.pos, cfg.box, leaf_size=leaf_size)
        rec, ropes = b["records"], b["ropes"]
        (m,) = b["meta"]
        idx = np.arange(rec.shape[0])
        assert np.all(ropes > idx) and np.all(ropes <= m["end"])
        assert ropes[m["root"]] == m["end"]  # the root's rope leaves the tree
        left = rec[:, 6].view(np.int32)
        right = rec[:, 7].view(np.int32)
        assert np.all((left < 0) | (left == idx + 1))  # an internal left child is the next record
        # an internal right child follows the left subtree; every run lies in the particle range
        assert np.all((right < 0) | (right > idx))
        covered = np.zeros(cfg.n, np.int64)
        for ref in np.concatenate([left[left < 0], right[right < 0]]):
            f, c = _run(ref)
            assert 1 <= c <= leaf_size
            covered[f:f + c] += 1
        assert np.all(covered == 1)  # runs partition the particles
