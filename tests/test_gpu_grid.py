"""The grid comparator (nlist_build_grid): the paper's comparison method on the
same GPU, with 1 to 32 cooperating lanes per particle.  Its lists equal the
oracle's row for row and the tree's count for count, for every lane count."""
import numpy as np
import pytest

import oracle
import paper_1901_08088_amd as Q
import workloads as W

from nlist_check import compare_rows, require_gpu, run_nlist

pytestmark = pytest.mark.gpu


def run_grid(cfg, max_nbr, grid=None, fill=-7, lanes=0):
    torch = require_gpu()
    n = cfg.n
    pos = torch.from_numpy(np.ascontiguousarray(cfg.pos)).cuda()
    nbr = torch.full((max(n, 1), max(max_nbr, 1)), fill, dtype=torch.int32, device="cuda")
    cnt = torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda")
    ovf = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    grid = Q.nlist_build_grid(pos, cfg.box, float(cfg.rcut[0, 0]), cfg.skin, max_nbr,
                              nbr if max_nbr > 0 else None, cnt, ovf, grid=grid, lanes=lanes)
    torch.cuda.synchronize()
    return grid, nbr.cpu().numpy()[:n, :max_nbr], cnt.cpu().numpy()[:n], int(ovf.item())


@pytest.mark.parametrize("make", [lambda: W.lj_fluid(4000), lambda: W.lj_fluid(30000, seed=30000, rho=0.6),
                                  lambda: W.wca_fluid(30000), lambda: W.spinodal(30000)])
def test_grid_rows_match_oracle_and_tree(make):
    cfg = make()
    tree, _, tcnt, tovf = run_nlist(cfg, 256)
    Q.qbvh_free(tree)
    first = None
    for lanes in (1, 2, 4, 8, 16, 32):
        print(f"[grid] {cfg.name} lanes {lanes}", flush=True)
        g, nbr, cnt, ovf = run_grid(cfg, 256, lanes=lanes)
        compare_rows(cfg, nbr, cnt, ovf, 256)
        assert np.array_equal(cnt, tcnt) and ovf == tovf
        # the order within a row is candidate order whatever the lane count
        if first is None:
            first = nbr
        else:
            assert np.array_equal(nbr, first)
        g.free()


@pytest.mark.parametrize("lanes", [1, 8, 32])
def test_grid_overflow_rows_keep_the_first_entries(lanes):
    # rows cut at widths that end inside a group's write
    cfg = W.lj_fluid(4000)
    _, full, fcnt, _ = run_grid(cfg, 256, lanes=lanes)
    for width in (5, 13):
        g, nbr, cnt, ovf = run_grid(cfg, width, lanes=lanes)
        assert ovf == 1 and np.array_equal(cnt, fcnt)
        assert np.array_equal(nbr, full[:, :width])
        g.free()


def test_grid_overflow_counts_only_and_reuse():
    cfg = W.lj_fluid(4000)
    g, nbr, cnt, ovf = run_grid(cfg, 8)
    assert ovf == 1
    compare_rows(cfg, nbr, cnt, ovf, 8)
    g, nbr, cnt, ovf = run_grid(cfg, 0, grid=g)
    compare_rows(cfg, nbr, cnt, ovf, 0)
    big = W.lj_fluid(30000, seed=30000, rho=0.6)  # a larger system through the same handle
    g, nbr, cnt, ovf = run_grid(big, 256, grid=g)
    compare_rows(big, nbr, cnt, ovf, 256)
    g.free()


def test_grid_geometry_errors():
    torch = require_gpu()
    pos = torch.zeros((10, 3), dtype=torch.float32, device="cuda")
    cnt = torch.empty(10, dtype=torch.int32, device="cuda")
    ovf = torch.empty(1, dtype=torch.int32, device="cuda")
    with pytest.raises(Q.QbvhError) as e:  # 2 r_list >= L
        Q.nlist_build_grid(pos, [6.0, 6.0, 6.0], 3.0, 0.1, 0, None, cnt, ovf)
    assert e.value.code == -2
    with pytest.raises(Q.QbvhError) as e:  # fewer than 3 cells on an axis
        Q.nlist_build_grid(pos, [7.0, 20.0, 20.0], 3.0, 0.1, 0, None, cnt, ovf)
    assert e.value.code == Q.ENOTSUP
    for lanes in (3, 64, -1):  # not a power of 2 below the wavefront width
        with pytest.raises(Q.QbvhError) as e:
            Q.nlist_build_grid(pos, [20.0, 20.0, 20.0], 3.0, 0.1, 0, None, cnt, ovf, lanes=lanes)
        assert e.value.code == Q.EINVAL


@pytest.mark.parametrize("lanes", [1, 8])
def test_grid_full_size_counts(lanes):
    require_gpu()
    cfg = W.lj_fluid(1_000_000)
    g, _, cnt, ovf = run_grid(cfg, 0, lanes=lanes)
    ocnt = oracle.neighbor_counts(cfg.pos, cfg.box, cfg.rcut, cfg.skin)
    assert np.array_equal(cnt.astype(np.int64), ocnt)
    g.free()
