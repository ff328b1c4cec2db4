"""Parity of the HIP path with the oracle, through the C interface.

Build steps are compared bit for bit with ``oracle/tree.py`` (keys, sort
permutation, radix tree, node boxes, quantized slots, per-tree metadata); the
neighbor lists are compared row by row with the oracle's definition
(counts equal, sorted rows equal, overflow semantics).  Sizes span several
sort tiles (4096 keys) and traversal workgroups with ragged tails.
"""
import numpy as np
import pytest

import oracle
import paper_1901_08088_amd as Q
import workloads as W
from oracle import tree as T

import layout_ref as LR

from nlist_check import compare_rows, export, require_gpu, run_nlist, to_dev

pytestmark = pytest.mark.gpu


def _step_parity(cfg, leaf_size=1, qbits=16, collapse_radius=0.0):
    torch = require_gpu()
    pos, types = to_dev(cfg)
    tree = Q.qbvh_build(pos, types, cfg.box, cfg.ntypes,
                        {"leaf_size": leaf_size, "qbits": qbits, "collapse_radius": collapse_radius})
    ref = LR.build_all(cfg.pos, cfg.box, types=cfg.types, ntypes=cfg.ntypes, leaf_size=leaf_size, qbits=qbits,
                       collapse_radius=collapse_radius)
    n = cfg.n
    info = Q.qbvh_info(tree)
    keys = export(tree, "keys", n, torch.int32).view(np.uint32)
    perm = export(tree, "perm", n, torch.int32).view(np.uint32)
    assert np.array_equal(keys, ref["sorted_keys"]), "sorted Morton keys"
    assert np.array_equal(perm, ref["perm"]), "sort permutation (stable)"
    srt = export(tree, "sorted", n, torch.float32, 4)
    assert np.array_equal(srt[:, :3].view(np.uint32), ref["sorted_pos"].view(np.uint32))
    assert np.array_equal(srt[:, 3].view(np.int32), ~ref["perm"].astype(np.int32))

    left = export(tree, "left", n, torch.int32)
    right = export(tree, "right", n, torch.int32)
    rf = export(tree, "range_f", n, torch.int32)
    rl = export(tree, "range_l", n, torch.int32)
    parent = export(tree, "parent", n, torch.int32)
    lparent = export(tree, "leaf_parent", n, torch.int32)
    blo = export(tree, "box_lo", n, torch.float32, 4)
    bhi = export(tree, "box_hi", n, torch.float32, 4)
    for t, (s, e) in enumerate(ref["segments"]):
        assert info["tree_start"][t] == s and info["tree_count"][t] == e - s
        ids = np.arange(s, max(e - 1, s))
        rstart = np.where(right[ids] < 0, ~right[ids], rf[np.clip(right[ids], 0, n - 1)])
        got = {(int(rf[i]), int(rl[i])): int(g) - 1 for i, g in zip(ids, rstart)}
        assert got == ref["trees"][t], f"radix tree of type {t}"
        for i in ids:  # parent links agree with the children
            for c in (left[i], right[i]):
                assert (lparent[~c] if c < 0 else parent[c]) == i
            lo, hi = ref["boxes"][t][(int(rf[i]), int(rl[i]))]
            assert np.array_equal(blo[i, :3], lo) and np.array_equal(bhi[i, :3], hi)
        if e - s >= 2:
            assert parent[s] == -1
    nrec = info["nrecords"]
    assert nrec == ref["records"].shape[0]
    rec = export(tree, "records", nrec, torch.int32, 8).view(np.uint32)
    ropes = export(tree, "ropes", nrec, torch.int32)
    mism = np.nonzero(np.any(rec != ref["records"], axis=1))[0]
    assert mism.size == 0, f"{mism.size} record mismatches, first {mism[:5].tolist()}"
    assert np.array_equal(ropes, ref["ropes"])
    for t, m in enumerate(ref["meta"]):
        if m["count"]:
            assert info["tree_root"][t] == m["root"] and info["tree_end"][t] == m["end"]
            assert np.array_equal(np.float32(info["root_lo"][t]), m["lo"])
            assert np.array_equal(np.float32(info["root_hi"][t]), m["hi"])
            assert info["h"][t] == m["h"]
    return tree


@pytest.mark.parametrize("n", [1, 2, 3, 4095, 4096, 4097, 3 * 4096 + 123])
def test_build_steps_sizes(n):
    pos, box = W.uniform(n, [11.0, 12.0, 13.0], seed=100 + n)
    _step_parity(W.Config(pos=pos, box=box, rcut=np.array([[2.0]], np.float32), skin=0.3))


@pytest.mark.parametrize("leaf_size,qbits", [(1, 10), (4, 16), (8, 12), (16, 16), (11, 10)])
def test_build_steps_lj4000(leaf_size, qbits):
    _step_parity(W.lj_fluid(4000), leaf_size=leaf_size, qbits=qbits)


@pytest.mark.parametrize("make,leaf_size,radius", [
    (lambda: W.lj_fluid(4000), 16, 3.4), (lambda: W.lj_fluid(4000), 16, 1.0), (lambda: W.lj_fluid(4000), 8, 2.0),
    (lambda: W.wca_fluid(9000, seed=5), 16, 1.52), (lambda: W.spinodal(12000, seed=6), 16, 3.4)])
def test_build_steps_cost_collapse(make, leaf_size, radius):
    # subtree collapse by the cost model: the same records as the layout helper
    _step_parity(make(), leaf_size=leaf_size, collapse_radius=radius)


def test_build_steps_cost_collapse_two_types():
    pos, box = W.uniform(6000, [14.0, 14.0, 14.0], seed=22)
    types = np.where(np.arange(6000) % 4 == 0, 1, 0).astype(np.int32)
    _step_parity(W.Config(pos=pos, box=box, rcut=np.ones((2, 2), np.float32), skin=0.2, types=types),
                 leaf_size=12, collapse_radius=1.2)


def test_build_steps_duplicate_codes():
    # many coincident and near-coincident points: equal Morton codes, ties by position
    rng = np.random.default_rng(5)
    base = rng.uniform(0, 9.0, size=(40, 3))
    pos = np.repeat(base, 50, axis=0) + rng.choice([0.0, 1e-4], size=(2000, 3))
    pos = W.wrap_f32(pos, np.full(3, 9.0, np.float32))
    _step_parity(W.Config(pos=pos, box=np.full(3, 9.0, np.float32), rcut=np.array([[1.0]], np.float32),
                          skin=0.1), leaf_size=2)


@pytest.mark.parametrize("clusters,leaf_size,radius", [(33, 4, 0.0), (70, 16, 0.0), (70, 16, 1.5)])
def test_build_steps_long_duplicate_runs(clusters, leaf_size, radius):
    # runs of 1000 coincident or near-coincident points (equal Morton codes,
    # ties by position) that cross first-level chunk borders and finish in
    # the upper levels (70 clusters: two levels), with and without the cost model
    rng = np.random.default_rng(9 + clusters)
    n = clusters * 1000
    base = rng.uniform(0, 30.0, size=(clusters, 3))
    pos = np.repeat(base, 1000, axis=0) + rng.choice([0.0, 1e-3], size=(n, 3))
    pos = W.wrap_f32(pos, np.full(3, 30.0, np.float32))
    _step_parity(W.Config(pos=pos, box=np.full(3, 30.0, np.float32), rcut=np.array([[1.0]], np.float32),
                          skin=0.1), leaf_size=leaf_size, collapse_radius=radius)


def test_build_steps_three_types_one_empty():
    pos, box = W.uniform(6000, [14.0, 14.0, 14.0], seed=21)
    types = np.where(np.arange(6000) % 5 == 0, 3, 0).astype(np.int32)
    rcut = np.ones((4, 4), np.float32)
    _step_parity(W.Config(pos=pos, box=box, rcut=rcut, skin=0.2, types=types))


# ------------------------------------------------------------------ neighbor lists

def test_lj4000_exact_lists_and_determinism():
    cfg = W.lj_fluid(4000)
    tree, nbr, cnt, ovf = run_nlist(cfg, 256)
    compare_rows(cfg, nbr, cnt, ovf, 256)
    _, nbr2, cnt2, ovf2 = run_nlist(cfg, 256, fill=-7)
    assert np.array_equal(nbr, nbr2) and np.array_equal(cnt, cnt2) and ovf == ovf2 == 0


@pytest.mark.parametrize("opts", [{"leaf_size": 1, "qbits": 10}, {"leaf_size": 4}, {"leaf_size": 8, "qbits": 12},
                                  {"leaf_size": 16}, {"leaf_size": 13, "qbits": 10, "block_size": 128},
                                  {"block_size": 64}, {"block_size": 192, "leaf_size": 2},
                                  {"collapse_radius": 3.4}, {"collapse_radius": 0.7, "leaf_size": 9}])
def test_lj4000_options(opts):
    cfg = W.lj_fluid(4000)
    _, nbr, cnt, ovf = run_nlist(cfg, 256, opts)
    compare_rows(cfg, nbr, cnt, ovf, 256)


@pytest.mark.parametrize("n,rho", [(50, 0.05), (777, 0.3), (12411, 0.85), (30000, 0.6), (40000, 0.85)])
def test_lattice_fluids(n, rho):
    # 50 to 30000 particles run 8 queries per wavefront, 40000 runs 16
    cfg = W.lj_fluid(n, seed=n, rho=rho)
    if 2 * 3.4 >= cfg.box.min():
        cfg = W.lj_fluid(n, seed=n, rho=rho, rc=1.0, skin=0.2)
    _, nbr, cnt, ovf = run_nlist(cfg, 256)
    compare_rows(cfg, nbr, cnt, ovf, 256)


def test_wca_fluid_rows():
    # short cutoff (rc = 2^(1/6)): about a dozen neighbors, small leaf boxes
    cfg = W.wca_fluid(30000)
    _, nbr, cnt, ovf = run_nlist(cfg, 64)
    compare_rows(cfg, nbr, cnt, ovf, 64)


def test_spinodal_rows():
    # liquid (0.75) and vapor (0.05) domains: wavefronts of very different work
    cfg = W.spinodal(30000)
    _, nbr, cnt, ovf = run_nlist(cfg, 256)
    compare_rows(cfg, nbr, cnt, ovf, 256)


def test_uniform_noncubic_box_scalar_rows():
    pos, box = W.uniform(9000, [17.0, 23.0, 29.0], seed=4)
    cfg = W.Config(pos=pos, box=box, rcut=np.array([[2.5]], np.float32), skin=0.3)
    _, nbr, cnt, ovf = run_nlist(cfg, 203)  # not a multiple of 4: scalar row stores
    compare_rows(cfg, nbr, cnt, ovf, 203)


def test_two_types_per_pair_radii():
    pos, box = W.uniform(8000, [18.0, 18.0, 18.0], seed=8)
    types = (np.arange(8000) % 7 == 0).astype(np.int32)
    rcut = np.array([[1.0, 2.0], [2.0, 3.0]], np.float32)
    cfg = W.Config(pos=pos, box=box, rcut=rcut, skin=0.4, types=types)
    _, nbr, cnt, ovf = run_nlist(cfg, 128)
    compare_rows(cfg, nbr, cnt, ovf, 128)


def test_disabled_type_pair_and_empty_type():
    pos, box = W.uniform(5000, [15.0, 15.0, 15.0], seed=9)
    types = np.where(np.arange(5000) % 3 == 0, 2, 0).astype(np.int32)
    rcut = np.array([[1.5, 0, 2.0], [0, 1.0, 0], [2.0, 0, 0.0]], np.float32)
    cfg = W.Config(pos=pos, box=box, rcut=rcut, skin=0.25, types=types)
    _, nbr, cnt, ovf = run_nlist(cfg, 64)
    compare_rows(cfg, nbr, cnt, ovf, 64)


@pytest.mark.parametrize("n", [5, 37, 300, 5000])
def test_four_types_uneven(n):
    # several types: every type's queries are spread over eight stretches,
    # smallest type first; types with fewer particles than stretches, an empty
    # type and equal type sizes must still give every row exactly once
    pos, box = W.uniform(n, [12.0, 12.0, 12.0], seed=n)
    k = np.arange(n)
    types = np.where(k % 9 == 0, 3, np.where(k % 9 == 1, 1, 0)).astype(np.int32)  # type 2 empty
    if n >= 4:
        types[-2:] = 1
    rcut = np.array([[1.5, 2.0, 1.0, 2.5], [2.0, 1.0, 0.0, 1.5], [1.0, 0.0, 2.0, 1.0], [2.5, 1.5, 1.0, 2.2]],
                    np.float32)
    cfg = W.Config(pos=pos, box=box, rcut=rcut, skin=0.3, types=types)
    for block in (64, 128, 256):
        _, nbr, cnt, ovf = run_nlist(cfg, 64, opts={"leaf_size": 4, "block_size": block})
        compare_rows(cfg, nbr, cnt, ovf, 64)


def test_overflow_keeps_true_counts():
    cfg = W.lj_fluid(4000)
    _, nbr, cnt, ovf = run_nlist(cfg, 8)
    assert ovf == 1
    compare_rows(cfg, nbr, cnt, ovf, 8)


@pytest.mark.parametrize("max_nbr", [1, 4, 12, 13, 20, 100])
def test_overflow_row_ends(max_nbr):
    """Rows cut at widths that end halfway through an 8-entry flush (4, 12,
    20 and 100 are 4 mod 8) and at widths that are not a multiple of 4 (the
    element-store path); with about 140 neighbours per particle every row
    overflows, so the last partial flush of each row is the one cut."""
    cfg = W.lj_fluid(4000, seed=7)
    _, nbr, cnt, ovf = run_nlist(cfg, max_nbr)
    assert ovf == 1
    compare_rows(cfg, nbr, cnt, ovf, max_nbr)


def test_counts_only():
    cfg = W.lj_fluid(4000)
    _, nbr, cnt, ovf = run_nlist(cfg, 0)
    assert ovf == 1
    compare_rows(cfg, nbr, cnt, ovf, 0)


def test_edge_positions_and_ties():
    L = 10.0
    pts = [[0.0, 0.0, 0.0], [np.nextafter(np.float32(L), np.float32(0)), 0.0, 0.0], [0.25, 0.25, 0.25],
           [1.0, 1.0, 1.0], [1.375, 1.5, 2.5], [5.0, 5.0, 5.0], [5.0, 5.0, 5.0], [5.0, 5.0, 6.625]]
    pos = np.array(pts, np.float32)
    cfg = W.Config(pos=pos, box=np.full(3, L, np.float32), rcut=np.array([[1.625]], np.float32), skin=0.0)
    _, nbr, cnt, ovf = run_nlist(cfg, 8)
    compare_rows(cfg, nbr, cnt, ovf, 8, method="brute")
    # the (3,4,12)/8 pair sits exactly at the cutoff and must be listed
    assert 4 in nbr[3, :cnt[3]] and 3 in nbr[4, :cnt[4]]


@pytest.mark.parametrize("n", [0, 1, 2])
def test_tiny_systems(n):
    pos = np.array([[1.0, 2.0, 3.0], [1.5, 2.0, 3.0]], np.float32)[:n]
    cfg = W.Config(pos=pos.reshape(-1, 3), box=np.full(3, 6.0, np.float32),
                   rcut=np.array([[1.0]], np.float32), skin=0.1)
    _, nbr, cnt, ovf = run_nlist(cfg, 4)
    assert ovf == 0
    if n:
        compare_rows(cfg, nbr, cnt, ovf, 4, method="brute")


def test_rebuild_in_place_and_grow():
    cfg_a = W.lj_fluid(3000, seed=1)
    cfg_b = W.lj_fluid(9000, seed=2)
    tree, nbr, cnt, ovf = run_nlist(cfg_a, 256)
    compare_rows(cfg_a, nbr, cnt, ovf, 256)
    tree, nbr, cnt, ovf = run_nlist(cfg_b, 256, tree=tree)
    compare_rows(cfg_b, nbr, cnt, ovf, 256)
    tree, nbr, cnt, ovf = run_nlist(cfg_a, 256, tree=tree)
    compare_rows(cfg_a, nbr, cnt, ovf, 256)


# -------------------------------------------------------------------- errors

def test_validation_rejects_out_of_box_and_bad_type():
    torch = require_gpu()
    cfg = W.lj_fluid(1000, seed=3)
    pos = cfg.pos.copy()
    pos[17, 1] = cfg.box[1]  # == L: outside [0, L)
    with pytest.raises(Q.QbvhError) as e:
        Q.qbvh_build(torch.from_numpy(pos).cuda(), None, cfg.box, 1, {"validate": 1})
    assert e.value.code == -1
    types = np.zeros(1000, np.int32)
    types[5] = 2
    with pytest.raises(Q.QbvhError):
        Q.qbvh_build(torch.from_numpy(cfg.pos).cuda(), torch.from_numpy(types).cuda(), cfg.box, 2,
                     {"validate": 1})
    Q.qbvh_build(torch.from_numpy(cfg.pos).cuda(), None, cfg.box, 1, {"validate": 1})


def test_geometry_and_radius_errors():
    torch = require_gpu()
    cfg = W.lj_fluid(1000, seed=3)  # L = 10.56
    tree = Q.qbvh_build(torch.from_numpy(cfg.pos).cuda(), None, cfg.box, 1)
    cnt = torch.zeros(1000, dtype=torch.int32, device="cuda")
    ovf = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(Q.QbvhError) as e:
        Q.nlist_build(tree, [[5.0]], 0.4, 0, None, cnt, ovf)
    assert e.value.code == -2
    with pytest.raises(Q.QbvhError) as e:
        Q.nlist_build(tree, [[1.0]], -0.1, 0, None, cnt, ovf)
    assert e.value.code == -1
