"""fp64 particle data (qbvh_build_f64, Section 2.2 and Figs. 4-7): the lists
equal the fp64 oracle's row for row, including pairs within 1e-13 to 1e-8 of
the cutoff that fp32 cannot resolve."""
import numpy as np
import pytest

import oracle
import paper_1901_08088_amd as Q
import workloads as W

from nlist_check import compare_rows, require_gpu, run_nlist

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("opts", [None, {"leaf_size": 1, "qbits": 10}, {"leaf_size": 8, "block_size": 128}])
def test_f64_lj_rows(opts):
    cfg = W.as_f64(W.lj_fluid(30000, seed=30000, rho=0.6), seed=1)
    _, nbr, cnt, ovf = run_nlist(cfg, 256, opts=opts)
    compare_rows(cfg, nbr, cnt, ovf, 256)


def test_f64_near_cutoff_pairs_decided_in_fp64():
    cfg = W.near_cutoff_pairs_f64(6000, 3000, 20.0, 1.7, seed=2)
    _, nbr, cnt, ovf = run_nlist(cfg, 64)
    rp, cols = compare_rows(cfg, nbr, cnt, ovf, 64)
    # the case is only meaningful if rounding to fp32 changes some rows
    rp32, cols32 = oracle.neighbor_lists(cfg.pos.astype(np.float32), cfg.box.astype(np.float32), cfg.rcut,
                                         cfg.skin)
    assert not (np.array_equal(rp, rp32) and np.array_equal(cols, cols32))


def test_f64_two_types_rows():
    c = W.colloid_solvent(n_total=3000, seed=7)
    cfg = W.as_f64(c, seed=3)
    _, nbr, cnt, ovf = run_nlist(cfg, 256)
    compare_rows(cfg, nbr, cnt, ovf, 256)


@pytest.mark.parametrize("opts", [None, {"leaf_size": 4}, {"leaf_size": 1, "qbits": 16}])
def test_f64_compact_type_near_cutoff(opts):
    # a type of 40 particles within 0.1 sigma in a box of edge 100: its tree's bins
    # (0.1 / 65535) are far below the shift of a pair's distance when both points
    # round to fp32 (up to sqrt(3) 2^-23 100); pairs at 2.5 (1 +- 1e-9..1e-6) from it
    cfg = W.compact_type_f64()
    _, nbr, cnt, ovf = run_nlist(cfg, 512, opts=opts)
    assert ovf == 0
    compare_rows(cfg, nbr, cnt, ovf, 512, method="brute")


def test_f64_rebuild_between_precisions_reuses_the_handle():
    c32 = W.lj_fluid(4000)
    c64 = W.as_f64(c32, seed=4)
    tree = None
    for cfg in (c32, c64, c32, c64):
        tree, nbr, cnt, ovf = run_nlist(cfg, 256, tree=tree)
        compare_rows(cfg, nbr, cnt, ovf, 256)
    Q.qbvh_free(tree)


def test_f64_validation_and_paper_mode():
    torch = require_gpu()
    cfg = W.as_f64(W.lj_fluid(4000), seed=5)
    pos = torch.from_numpy(cfg.pos.copy()).cuda()
    tree = Q.qbvh_build(pos, None, cfg.box, 1, {"validate": 1})
    n = cfg.n
    nbr = torch.empty((n, 256), dtype=torch.int32, device="cuda")
    cnt = torch.empty(n, dtype=torch.int32, device="cuda")
    ovf = torch.empty(1, dtype=torch.int32, device="cuda")
    with pytest.raises(Q.QbvhError) as e:
        Q.nlist_build_ex(tree, cfg.rcut, cfg.skin, 256, Q.LIST_PAPER, nbr, cnt, ovf)
    assert e.value.code == Q.ENOTSUP
    bad = cfg.pos.copy()
    bad[17, 1] = cfg.box[1]  # x == L is outside [0, L)
    with pytest.raises(Q.QbvhError) as e:
        Q.qbvh_build(torch.from_numpy(bad).cuda(), None, cfg.box, 1, {"validate": 1}, tree=tree)
    assert e.value.code == Q.EINVAL
    Q.qbvh_free(tree)


def test_f64_full_size_counts_and_sampled_rows():
    torch = require_gpu()
    cfg = W.as_f64(W.lj_fluid(1_000_000), seed=6)
    n = cfg.n
    pos = torch.from_numpy(cfg.pos).cuda()
    tree = Q.qbvh_build(pos, None, cfg.box, 1, None)
    nbr = torch.empty((n, 256), dtype=torch.int32, device="cuda")
    cnt = torch.empty(n, dtype=torch.int32, device="cuda")
    ovf = torch.empty(1, dtype=torch.int32, device="cuda")
    Q.nlist_build(tree, cfg.rcut, cfg.skin, 256, nbr, cnt, ovf)
    torch.cuda.synchronize()
    gcnt = cnt.cpu().numpy().astype(np.int64)
    ocnt = oracle.neighbor_counts(cfg.pos, cfg.box, cfg.rcut, cfg.skin)
    assert np.array_equal(gcnt, ocnt)
    rng = np.random.default_rng(8)
    sample = np.sort(rng.choice(n, 2000, replace=False))
    rows = nbr[torch.from_numpy(sample).cuda()].cpu().numpy()
    rp, cols = oracle.neighbor_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, queries=sample)
    for q, i in enumerate(sample):
        assert sorted(rows[q, :gcnt[i]].tolist()) == cols[rp[q]:rp[q + 1]].tolist(), i
    Q.qbvh_free(tree)
