"""Step-by-step oracle of the tree the method builds.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every function here is
written from its definition, with plain NumPy and Python loops, for the small
inputs the tests use.  It shares nothing with the HIP library.

Steps, in the paper's order (Section 2.1, "Bounding volume hierarchy";
Section 2.2, "Compressed BVH"):

1. ``morton_keys``   -- box split into 2^10 - 1 bins per axis, 10-bit bin
                         coordinates interleaved into a 30-bit Morton code.
2. ``sort_keys``     -- sort along the Z-order curve (stable, so equal codes
                         keep index order; Section 3 asks for determinism).
3. ``radix_tree``    -- Karras's binary radix tree over the sorted codes
                         (N - 1 internal nodes with exactly two children);
                         equal codes are told apart by their sorted position,
                         which is Karras's own tie rule.
4. ``node_boxes``    -- axis-aligned box of every internal node, i.e. the
                         min/max over the particles below it (what the
                         bottom-up fit computes).
5. ``grid_spacing`` and ``quantize_box`` -- the root-node box of a tree
                         divided into 2^b - 1 bins along each axis; a box's
                         lower bounds rounded down and upper bounds rounded up
                         onto that grid (Section 2.2; Section 3 for the
                         directed rounding).

How a quantized tree is laid out in memory (node size, child and rope
encoding) is a design choice of an implementation, not part of the method;
it is not defined here.

Readings where the paper is silent (listed again in the design notes):
- One tree per particle type; the type is stored above the 30-bit code
  (bits 30-31) so one sort groups the types.
- An axis along which the root-node box has no extent (all of the tree's
  particles share that coordinate) still gets a grid: its extent is floored
  at 2^-24 of the largest periodic box edge.
"""
from __future__ import annotations

import numpy as np

MORTON_BITS = 10
MORTON_MAX = (1 << MORTON_BITS) - 1  # 1023 bins per axis


def morton_keys(pos, box, types=None) -> np.ndarray:
    """30-bit Morton code per particle, type in bits 30-31 (uint32).

    Per axis the bin is floor(x * (1023 / L)) in fp64, clamped to [0, 1023];
    bit k of the x, y and z bins goes to code bits 3k, 3k+1 and 3k+2.
    """
    pos = np.asarray(pos, dtype=np.float32).reshape(-1, 3)
    L = np.asarray(box, dtype=np.float32).astype(np.float64)
    scale = float(MORTON_MAX) / L
    b = np.floor(pos.astype(np.float64) * scale)
    b = np.clip(b, 0, MORTON_MAX).astype(np.uint32)
    code = np.zeros(pos.shape[0], dtype=np.uint32)
    for k in range(MORTON_BITS):
        for axis in range(3):
            bit = (b[:, axis] >> np.uint32(k)) & np.uint32(1)
            code |= bit << np.uint32(3 * k + axis)
    if types is not None:
        code |= np.asarray(types, dtype=np.uint32) << np.uint32(30)
    return code


def sort_keys(keys):
    """Stable ascending sort: returns (sorted keys, permutation)."""
    perm = np.argsort(keys, kind="stable").astype(np.uint32)
    return np.asarray(keys)[perm], perm


def segments(sorted_keys, ntypes: int):
    """Half-open sorted-index range [s, e) of each type's tree."""
    t = (np.asarray(sorted_keys, dtype=np.uint32) >> np.uint32(30)).astype(np.int64)
    bounds = []
    for ty in range(ntypes):
        idx = np.nonzero(t == ty)[0]
        if idx.size == 0:
            s = int(np.searchsorted(t, ty))
            bounds.append((s, s))
        else:
            bounds.append((int(idx[0]), int(idx[-1]) + 1))
    return bounds


def radix_tree(sorted_keys, s: int, e: int) -> dict:
    """Binary radix tree over sorted positions [s, e): {(f, l): gamma}.

    The augmented key of position k is (key_k << 32) | k.  A node covering
    [f, l] splits at the highest bit in which the augmented keys of f and l
    differ: its left child covers [f, gamma], where gamma is the last position
    whose augmented key has a 0 in that bit, and its right child
    [gamma + 1, l].  Ranges of one position are leaves (not stored).
    """
    nodes = {}
    if e - s < 2:
        return nodes
    a = (np.asarray(sorted_keys[s:e], dtype=np.uint64) << np.uint64(32)) | \
        np.arange(s, e, dtype=np.uint64)
    stack = [(s, e - 1)]
    while stack:
        f, l = stack.pop()
        x = int(a[f - s]) ^ int(a[l - s])
        bit = x.bit_length() - 1
        bits = (a[f - s:l - s + 1] >> np.uint64(bit)) & np.uint64(1)
        gamma = f + int(np.count_nonzero(bits == 0)) - 1
        nodes[(f, l)] = gamma
        if gamma > f:
            stack.append((f, gamma))
        if gamma + 1 < l:
            stack.append((gamma + 1, l))
    return nodes


def node_boxes(sorted_pos, nodes: dict) -> dict:
    """Box of each internal node: component-wise min and max over its particles."""
    p = np.asarray(sorted_pos, dtype=np.float32).reshape(-1, 3)
    return {(f, l): (p[f:l + 1].min(axis=0), p[f:l + 1].max(axis=0)) for (f, l) in nodes}


def grid_spacing(lo, hi, box, qbits: int) -> np.ndarray:
    """Bin width along each axis of the grid over the root-node box [lo, hi]:
    h_d = extent_d / (2^b - 1) in fp64, with extent_d floored at 2^-24 of the
    largest periodic box edge (fp64 array of 3)."""
    floor_ext = float(np.max(np.asarray(box, dtype=np.float32).astype(np.float64))) * 2.0 ** -24
    h = np.empty(3, np.float64)
    for d in range(3):
        ext = float(np.float64(hi[d])) - float(np.float64(lo[d]))
        h[d] = max(ext, floor_ext) / float((1 << qbits) - 1)
    return h


def quantize_box(lo, hi, root_lo, h, qbits: int):
    """Grid coordinates of a box: lower bounds rounded down, upper bounds up.

    q_lo = floor((lo - root_lo) / h_d), q_hi = ceil((hi - root_lo) / h_d),
    both evaluated in fp64 and clamped to [0, 2^qbits - 1].  ``h`` is the bin
    width of each axis (a scalar is taken for all three).
    """
    qmax = (1 << qbits) - 1
    hd = np.broadcast_to(np.asarray(h, dtype=np.float64), (3,))
    qlo, qhi = [], []
    for d in range(3):
        tl = (float(np.float64(lo[d])) - float(np.float64(root_lo[d]))) / float(hd[d])
        th = (float(np.float64(hi[d])) - float(np.float64(root_lo[d]))) / float(hd[d])
        qlo.append(int(min(max(np.floor(tl), 0), qmax)))
        qhi.append(int(min(max(np.ceil(th), 0), qmax)))
    return qlo, qhi


def build_steps(pos, box, types=None, ntypes: int = 1):
    """Run steps 1-4; returns a dict with each intermediate result."""
    keys = morton_keys(pos, box, types)
    skeys, perm = sort_keys(keys)
    p = np.asarray(pos, dtype=np.float32).reshape(-1, 3)[perm]
    segs = segments(skeys, ntypes)
    trees = [radix_tree(skeys, s, e) for (s, e) in segs]
    boxes = [node_boxes(p, tr) for tr in trees]
    return dict(keys=keys, sorted_keys=skeys, perm=perm, sorted_pos=p, segments=segs,
                trees=trees, boxes=boxes)
