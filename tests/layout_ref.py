"""Expected memory layout of the library's quantized tree, for the step parity
tests.

This is a test helper, not part of the oracle: the paper defines the steps of
the build (``oracle/tree.py``), while the layout below -- two-wide 32-byte
records, an isotropic grid, 16-bit bound fields, particle runs of at most
``leaf_size`` and the run encoding -- is this library's own design.  It takes
the tree, the boxes and the outward quantization from the oracle and only
arranges them.  The layout itself is pinned by ``test_tree_oracle_pins.py``,
which runs the paper's stackless traversal (Algorithm 1) over these records on
the CPU and must reproduce the oracle's brute-force neighbor lists.

Layout:
- Bin width: one isotropic h = (largest edge of the root-node box) / (2^b - 1)
  for all three axes (with that edge floored like the oracle's per-axis
  extents).  The traversal then tests a sphere in grid units with a single
  squared radius.
- Records in depth-first preorder per type tree, one per internal node whose
  particle range is longer than ``leaf_size``:
    words 0-2: box of the left child, w_d = q_lo_d | (q_hi_d << 16)
    words 3-5: box of the right child, same packing
    word 6/7:  left/right child: the record index (>= 0), or the particle run
               ~((first << 4) | (count - 1)) when the child holds at most
               ``leaf_size`` particles
  The left child's record is the next record; ropes[v] is the record after
  v's subtree.  A tree of at most ``leaf_size`` particles has no record: its
  root is a run.
- Subtree collapse by cost (``collapse_radius`` R > 0): a node of at most
  ``leaf_size`` particles becomes a run when
      count V(node) <= 4 V(node) + F(left) + F(right),
  F(particle) = V(point), F(node) = the smaller side, with V the node box's
  volume grown by R (Steiner's formula), all in fp32 in the library's order;
  a node keeps a record unless it or an ancestor became a run.
"""
from __future__ import annotations

import numpy as np

from oracle import tree as T


def iso_spacing(lo, hi, box, qbits: int) -> float:
    """The library's isotropic bin width: the largest of the per-axis widths."""
    return float(np.max(T.grid_spacing(lo, hi, box, qbits)))


def collapse_flags(tree: dict, boxes: dict, leaf_size: int, collapse_radius: float) -> dict:
    """{(f, l): True} for the internal nodes that become runs under the cost model."""
    f32 = np.float32
    R = float(np.float32(collapse_radius))
    pi = 3.141592653589793
    k2R, kPiR2, kVball = f32(2.0 * R), f32(pi * R * R), f32(4.0 / 3.0 * pi * R * R * R)
    F, coll = {}, {}
    for (f, l) in sorted(tree, key=lambda fl: fl[1] - fl[0]):  # children before parents
        g = tree[(f, l)]
        lo, hi = boxes[(f, l)]
        a, b, c = f32(hi[0] - lo[0]), f32(hi[1] - lo[1]), f32(hi[2] - lo[2])
        ab, bc, ca = f32(a * b), f32(b * c), f32(c * a)
        v = f32(f32(f32(f32(ab * c) + f32(k2R * f32(f32(ab + bc) + ca))) + f32(kPiR2 * f32(f32(a + b) + c))) + kVball)
        fc = [kVball if cf == cl else abs(F[(cf, cl)]) for (cf, cl) in ((f, g), (g + 1, l))]
        count = l - f + 1
        leafc = f32(f32(count) * v)
        split = f32(f32(f32(4.0) * v) + f32(fc[0] + fc[1]))
        coll[(f, l)] = bool(count <= leaf_size and leafc <= split)
        F[(f, l)] = f32(-leafc) if coll[(f, l)] else split
    return coll


def run_ref(first: int, count: int) -> int:
    """Reference to the particle run [first, first + count) (negative int32)."""
    return ~((first << 4) | (count - 1))


def record_layout(sorted_pos, sorted_keys, ntypes: int, box, leaf_size: int = 1, qbits: int = 16,
                  collapse_radius: float = 0.0):
    """Two-wide quantized records for all types' trees.

    Returns (records uint32 [M, 8], ropes int32 [M], meta list); ``meta[t]``
    holds the tree's root reference, one past its last record, its root box
    and its bin width.
    """
    assert 1 <= leaf_size <= 16
    p = np.asarray(sorted_pos, dtype=np.float32).reshape(-1, 3)
    records, ropes, meta = [], [], []
    for t, (s, e) in enumerate(T.segments(sorted_keys, ntypes)):
        first = len(records)
        if e == s:
            meta.append(dict(start=s, count=0, root=0, end=first, lo=None, hi=None, h=1.0))
            continue
        tree = T.radix_tree(sorted_keys, s, e)
        rlo = p[s:e].min(axis=0)
        rhi = p[s:e].max(axis=0)
        h = iso_spacing(rlo, rhi, box, qbits)
        if collapse_radius > 0:
            coll = collapse_flags(tree, T.node_boxes(p, tree), leaf_size, collapse_radius)
            is_run = lambda f, l: f == l or coll[(f, l)]  # noqa: E731
        else:
            is_run = lambda f, l: l - f + 1 <= leaf_size  # noqa: E731
        if is_run(s, e - 1):
            meta.append(dict(start=s, count=e - s, root=run_ref(s, e - s), end=first, lo=rlo, hi=rhi, h=h))
            continue

        def child_box(f, l):
            qlo, qhi = T.quantize_box(p[f:l + 1].min(axis=0), p[f:l + 1].max(axis=0), rlo, h, qbits)
            return [qlo[d] | (qhi[d] << 16) for d in range(3)]

        def emit(f, l):
            """Record of node [f, l] in preorder: itself, then its left and right subtrees."""
            idx = len(records)
            g = tree[(f, l)]
            kids = [(f, g), (g + 1, l)]
            records.append(child_box(*kids[0]) + child_box(*kids[1]) + [0, 0])
            ropes.append(-1)
            for side, (cf, cl) in enumerate(kids):
                if not is_run(cf, cl):
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


def build_all(pos, box, types=None, ntypes: int = 1, leaf_size: int = 1, qbits: int = 16,
              collapse_radius: float = 0.0):
    """The oracle's build steps plus the library's record layout."""
    b = T.build_steps(pos, box, types, ntypes)
    records, ropes, meta = record_layout(b["sorted_pos"], b["sorted_keys"], ntypes, box, leaf_size, qbits,
                                         collapse_radius)
    b.update(records=records, ropes=ropes, meta=meta)
    return b
