"""The library finds the radix tree bottom-up, together with the fit, instead
of by Karras's top-down searches: a node [l, r] is bounded by the splits l - 1
and r (split k weighs the common prefix length of the augmented keys at k and
k + 1, -1 between trees), its parent's split is the heavier of the two, a left
child takes its range end as id and a right child or a root its range start,
and at each split the first of the two children to arrive stops while the
second merges both.  The climb runs in chunks of sorted positions and levels
of chunks, each chunk passing on a frontier of finished nodes whose parent did
not finish in it.

This CPU model of that construction (the same rules, in plain Python, with
every interleaving of the climbs drawn at random) must produce the oracle's
top-down radix tree (Section 2.1) node for node, ids included, on random keys
with duplicates, several type trees and several systems, for chunk sizes and
fanouts small enough that every level and frontier rule is exercised; the
frontier of a chunk must stay within the two border chains.
"""
import random

import numpy as np
import pytest

from oracle import tree as T

EMPTY, DONE = -1, -2


def _weights(keys, cuts):
    n = len(keys)
    d = []
    for k in range(n):
        if k + 1 >= n or k in cuts or (int(keys[k]) ^ int(keys[k + 1])) >> 30:
            d.append(-1)
        elif keys[k] != keys[k + 1]:
            d.append(32 - (int(keys[k]) ^ int(keys[k + 1])).bit_length())
        else:
            d.append(64 - (k ^ (k + 1)).bit_length())
    return d


def _child_at(g, e):
    if e <= g:
        return ~g if e == g else g
    return ~(g + 1) if e == g + 1 else g + 1


def climb_tree(keys, cuts, chunk0, fanout, rng, cap=160, weights=_weights):
    """Node arrays (by id) from the chunked bottom-up climb."""
    n = len(keys)
    D = weights(keys, cuts)
    out = {k: {} for k in ("rf", "rl", "left", "right", "parent", "leaf_parent")}
    slot = {}

    def dl_of(l):
        return D[l - 1] if l > 0 else -1

    def write(K, l, r, cl, cr):
        assert K not in out["rf"], f"node {K} written twice"
        out["rf"][K], out["rl"][K], out["left"][K], out["right"][K] = l, r, cl, cr
        for c in (cl, cr):
            if c < 0:
                out["leaf_parent"][~c] = K
            else:
                out["parent"][c] = K

    def climb(l, r, fresh, c0, c1, front, pend, cl=0, cr=0):
        dl, dr = dl_of(l), D[r]
        for _ in range(200):
            leaf, root, goes_left = l == r, dl < 0 and dr < 0, dr > dl
            K = ~l if leaf else (r if goes_left and not root else l)
            if fresh and not leaf:
                write(K, l, r, cl, cr)
            if root:
                out["leaf_parent" if leaf else "parent"][l if leaf else K] = -1
                return
            g = r if goes_left else l - 1
            if g < c0 or g >= c1 - 1:
                front.append(K)
                return
            e = slot.get(g, EMPTY)
            slot[g] = l if goes_left else r
            if e == EMPTY:
                pend.append(g)
                return
            slot[g] = DONE
            sib = _child_at(g, e)
            if goes_left:
                r, dr, cl, cr = e, D[e], K, sib
            else:
                l, dl, cl, cr = e, dl_of(e), sib, K
            fresh = True
        raise AssertionError("climb deeper than the tree")

    def finish(front, pend):
        for g in pend:
            if slot[g] >= 0:
                front.append(_child_at(g, slot[g]))
            slot[g] = EMPTY
        assert len(front) <= cap
        return front

    chunk, fronts = chunk0, []
    for c0 in range(0, n, chunk):
        c1 = min(c0 + chunk, n)
        front, pend = [], []
        order = list(range(c0, c1))
        rng.shuffle(order)
        for i in order:
            climb(i, i, True, c0, c1, front, pend)
        fronts.append(finish(front, pend))
    while chunk < n:
        chunk *= fanout
        new = []
        for b, c0 in enumerate(range(0, n, chunk)):
            c1 = min(c0 + chunk, n)
            entries = [c for f in fronts[b * fanout:(b + 1) * fanout] for c in f]
            rng.shuffle(entries)
            front, pend = [], []
            for c in entries:
                l, r = (~c, ~c) if c < 0 else (out["rf"][c], out["rl"][c])
                climb(l, r, False, c0, c1, front, pend)
            new.append(finish(front, pend))
        fronts = new
    assert all(not f for f in fronts), "a frontier left after the last level"
    return out


def karras_arrays(keys, segs):
    """The oracle's top-down tree in the same arrays, Karras's ids."""
    ref = {k: {} for k in ("rf", "rl", "left", "right", "parent", "leaf_parent")}
    for s, e in segs:
        if e - s == 1:
            ref["leaf_parent"][s] = -1
        if e - s < 2:
            continue
        nodes = T.radix_tree(keys, s, e)
        ids = {(s, e - 1): s}
        ref["parent"][s] = -1
        for (f, l), g in sorted(nodes.items(), key=lambda x: x[0][0] - x[0][1]):
            K = ids[(f, l)]
            cl = g if g > f else ~f
            cr = g + 1 if g + 1 < l else ~l
            if g > f:
                ids[(f, g)] = g
            if g + 1 < l:
                ids[(g + 1, l)] = g + 1
            ref["rf"][K], ref["rl"][K], ref["left"][K], ref["right"][K] = f, l, cl, cr
            for c in (cl, cr):
                if c < 0:
                    ref["leaf_parent"][~c] = K
                else:
                    ref["parent"][c] = K
    return ref


def _case(rng):
    n = rng.choice([1, 2, 3, 5, 17, 64, 100, 257, 700])
    ntypes = rng.choice([1, 1, 2, 4])
    nsys = rng.choice([1, 1, 3]) if n > 3 else 1
    bounds = [0, n] if nsys == 1 else [0] + sorted(rng.sample(range(1, n), nsys - 1)) + [n]
    kind = rng.choice(["random", "duplicates", "few"])
    keys = []
    for a, b in zip(bounds[:-1], bounds[1:]):
        if kind == "random":
            body = [rng.getrandbits(30) for _ in range(b - a)]
        elif kind == "duplicates":
            body = [rng.getrandbits(5) for _ in range(b - a)]
        else:
            body = [rng.choice([5, 5, 9, 1 << 20]) for _ in range(b - a)]
        keys += sorted(k | (rng.randrange(ntypes) << 30) for k in body)
    cuts = {b - 1 for b in bounds[1:-1]}
    segs = []
    for a, b in zip(bounds[:-1], bounds[1:]):
        s = a
        for k in range(a, b):
            if k + 1 == b or (keys[k] >> 30) != (keys[k + 1] >> 30):
                segs.append((s, k + 1))
                s = k + 1
    return np.array(keys, np.uint32), cuts, segs


@pytest.mark.parametrize("seed", range(6))
def test_climb_builds_the_oracle_tree(seed):
    rng = random.Random(1901 + seed)
    for _ in range(40):
        keys, cuts, segs = _case(rng)
        chunk0, fanout = rng.choice([2, 4, 8, 16, 1024]), rng.choice([2, 3, 32])
        got = climb_tree(keys, cuts, chunk0, fanout, rng)
        ref = karras_arrays(keys, segs)
        for k in ref:
            assert got[k] == ref[k], (k, chunk0, fanout, len(keys))


def test_planted_parent_rule_fails():
    # taking the lighter bounding split as the parent's split must not pass
    rng = random.Random(7)
    keys = np.array(sorted(rng.getrandbits(30) for _ in range(64)), np.uint32)
    ref = karras_arrays(keys, [(0, 64)])

    def lighter_first(k, c):  # the weights negated: the lighter split now wins
        return [-d if d >= 0 else d for d in _weights(k, c)]

    try:
        got = climb_tree(keys, set(), 8, 2, rng, weights=lighter_first)
    except AssertionError:
        return  # the climb itself broke down
    assert got["left"] != ref["left"] or got["parent"] != ref["parent"]
