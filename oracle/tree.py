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
5. ``record_layout`` -- quantized nodes in a stackless, rope-linked order:
                         bounds snapped to a grid over the root-node box,
                         lower bounds rounded down and upper bounds up, and a
                         rope per node giving the next node to test when
                         nothing below it needs visiting.

Readings where the paper is silent (listed again in the design notes):
- One tree per particle type; the type is stored above the 30-bit code
  (bits 30-31) so one sort groups the types.
- The grid is isotropic: one bin width h = extent / (2^b - 1) for all axes,
  where extent is the largest edge of the root-node box (floored at 2^-24 of
  the largest periodic box edge so that a tree of coincident points still has
  a usable grid).  Bounds are stored in 16-bit fields for any b <= 16.
- Nodes are laid out as two-wide records in depth-first preorder: the record
  of an internal node holds the quantized boxes of its two children and a
  reference to each (the record of an internal child, or a run of at most
  ``leaf_size`` consecutive sorted particles: a subtree that small is not
  split further), and a separate array holds its rope (the record after its
  subtree).  The left child's record is the next record.  Testing both child
  boxes in the parent halves the chain of dependent node loads of a walk.
- A particle-run reference is ~((first << 4) | (count - 1)), negative; a
  record reference is the record index, non-negative.  A tree of at most
  ``leaf_size`` particles has no record: its root is a run.
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


def grid_spacing(lo, hi, box, qbits: int) -> float:
    """Isotropic bin width over the root-node box [lo, hi] (fp64)."""
    ext = max(float(np.float64(hi[d]) - np.float64(lo[d])) for d in range(3))
    floor_ext = float(np.max(np.asarray(box, dtype=np.float32).astype(np.float64))) * 2.0 ** -24
    ext = max(ext, floor_ext)
    return ext / float((1 << qbits) - 1)


def quantize_box(lo, hi, root_lo, h: float, qbits: int):
    """Grid coordinates of a box: lower bounds rounded down, upper bounds up.

    q_lo = floor((lo - root_lo) / h), q_hi = ceil((hi - root_lo) / h), both
    evaluated in fp64 and clamped to [0, 2^qbits - 1].
    """
    qmax = (1 << qbits) - 1
    qlo, qhi = [], []
    for d in range(3):
        tl = (float(np.float64(lo[d])) - float(np.float64(root_lo[d]))) / h
        th = (float(np.float64(hi[d])) - float(np.float64(root_lo[d]))) / h
        qlo.append(int(min(max(np.floor(tl), 0), qmax)))
        qhi.append(int(min(max(np.ceil(th), 0), qmax)))
    return qlo, qhi


def run_ref(first: int, count: int) -> int:
    """Reference to the particle run [first, first + count) (negative int32)."""
    return ~((first << 4) | (count - 1))


def record_layout(sorted_pos, sorted_keys, ntypes: int, box, leaf_size: int = 1, qbits: int = 16):
    """Two-wide quantized records for all types' trees.

    Returns (records uint32 [M, 8], ropes int32 [M], meta list).  Record of
    internal node v with children a (left) and b (right):
      words 0-2: box of a, w_d = q_lo_d | (q_hi_d << 16) for d = x, y, z
      words 3-5: box of b, same packing
      word 6:    reference to a;  word 7: reference to b
    ropes[v] = index of the record that follows v's subtree.  Trees follow
    each other in type order; ``meta[t]`` holds the tree's root reference,
    one past its last record, its root box and its grid spacing.
    """
    assert 1 <= leaf_size <= 16
    p = np.asarray(sorted_pos, dtype=np.float32).reshape(-1, 3)
    records, ropes, meta = [], [], []
    for t, (s, e) in enumerate(segments(sorted_keys, ntypes)):
        first = len(records)
        if e == s:
            meta.append(dict(start=s, count=0, root=0, end=first, lo=None, hi=None, h=1.0))
            continue
        tree = radix_tree(sorted_keys, s, e)
        rlo = p[s:e].min(axis=0)
        rhi = p[s:e].max(axis=0)
        h = grid_spacing(rlo, rhi, box, qbits)
        if e - s <= leaf_size:
            meta.append(dict(start=s, count=e - s, root=run_ref(s, e - s), end=first, lo=rlo, hi=rhi, h=h))
            continue

        def child_box(f, l):
            qlo, qhi = quantize_box(p[f:l + 1].min(axis=0), p[f:l + 1].max(axis=0), rlo, h, qbits)
            return [qlo[d] | (qhi[d] << 16) for d in range(3)]

        def emit(f, l):
            """Record of node [f, l] in preorder: itself, then its left and right subtrees."""
            idx = len(records)
            g = tree[(f, l)]
            kids = [(f, g), (g + 1, l)]
            records.append(child_box(*kids[0]) + child_box(*kids[1]) + [0, 0])
            ropes.append(-1)
            for side, (cf, cl) in enumerate(kids):
                if cl - cf + 1 > leaf_size:
                    ref = emit(cf, cl)
                else:
                    ref = run_ref(cf, cl - cf + 1)
                records[idx][6 + side] = ref & 0xFFFFFFFF
            ropes[idx] = len(records)
            return idx

        emit(s, e - 1)
        meta.append(dict(start=s, count=e - s, root=first, end=len(records), lo=rlo, hi=rhi, h=h))
    arr = np.array(records, dtype=np.uint32).reshape(-1, 8) if records else np.zeros((0, 8), np.uint32)
    return arr, np.array(ropes, dtype=np.int32), meta


def build_all(pos, box, types=None, ntypes: int = 1, leaf_size: int = 1, qbits: int = 16):
    """Run every step; returns a dict with each intermediate result."""
    keys = morton_keys(pos, box, types)
    skeys, perm = sort_keys(keys)
    p = np.asarray(pos, dtype=np.float32).reshape(-1, 3)[perm]
    segs = segments(skeys, ntypes)
    trees = [radix_tree(skeys, s, e) for (s, e) in segs]
    boxes = [node_boxes(p, tr) for tr in trees]
    records, ropes, meta = record_layout(p, skeys, ntypes, box, leaf_size, qbits)
    return dict(keys=keys, sorted_keys=skeys, perm=perm, sorted_pos=p, segments=segs,
                trees=trees, boxes=boxes, records=records, ropes=ropes, meta=meta)
