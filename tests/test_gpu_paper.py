"""Paper-mode lists (Section 2.3: leaf-box overlap, no distance check) on the
GPU against the paper-mode oracle: every row lies between the oracle's lists
without and with a small radius pad (the kernel's own rounding pad of 0.02
bins lies inside), contains the exact row, and the false positives match the
closed form."""
import numpy as np
import pytest

import oracle
import paper_1901_08088_amd as Q
import workloads as W
from oracle import paper as P

from nlist_check import require_gpu, to_dev

pytestmark = pytest.mark.gpu


def _paper_rows(cfg, opts, max_nbr=512):
    torch = require_gpu()
    pos, types = to_dev(cfg)
    tree = Q.qbvh_build(pos, types, cfg.box, cfg.ntypes, opts)
    n = cfg.n
    nbr = torch.full((n, max_nbr), -7, dtype=torch.int32, device="cuda")
    cnt = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    ovf = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    Q.nlist_build_ex(tree, cfg.rcut, cfg.skin, max_nbr, Q.LIST_PAPER, nbr, cnt, ovf)
    torch.cuda.synchronize()
    Q.qbvh_free(tree)
    return nbr.cpu().numpy(), cnt.cpu().numpy(), int(ovf.item())


def _check(cfg, qbits, nbr, cnt, ovf, max_nbr, queries=None):
    """Rows (all, or ``queries``) inside the oracle bracket; returns the mean false
    positives per particle over the checked rows."""
    assert ovf == 0 and cnt.max() <= max_nbr
    rows = np.arange(cfg.n) if queries is None else np.asarray(queries)
    lo_rp, lo_c = P.paper_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, types=cfg.types, qbits=qbits,
                                queries=queries)
    hi_rp, hi_c = P.paper_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, types=cfg.types, qbits=qbits, pad=0.05,
                                queries=queries)
    ex_rp, ex_c = oracle.neighbor_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, types=cfg.types, queries=queries)
    for k, i in enumerate(rows):
        row = nbr[i, :cnt[i]]
        got = set(row.tolist())
        assert len(got) == cnt[i], f"row {i} has duplicates"
        assert set(lo_c[lo_rp[k]:lo_rp[k + 1]].tolist()) <= got, f"row {i} misses a paper-mode neighbor"
        assert got <= set(hi_c[hi_rp[k]:hi_rp[k + 1]].tolist()), f"row {i} lists a particle beyond the pad"
        assert set(ex_c[ex_rp[k]:ex_rp[k + 1]].tolist()) <= got
    return float(cnt[rows].sum() - (ex_rp[-1])) / rows.size


@pytest.mark.parametrize("leaf,qbits", [(1, 10), (4, 10), (8, 10), (8, 16), (3, 8), (16, 10), (12, 10)])
def test_paper_mode_lj4000(leaf, qbits):
    cfg = W.lj_fluid(4000)
    nbr, cnt, ovf = _paper_rows(cfg, {"leaf_size": leaf, "qbits": qbits})
    fp = _check(cfg, qbits, nbr, cnt, ovf, 512)
    print(f"[paper] leaf {leaf} bits {qbits}: {fp:.3f} false positives per particle", flush=True)


def test_paper_mode_false_positives_ideal_gas():
    n, rho = 6000, 0.85
    box = np.full(3, (n / rho) ** (1.0 / 3.0), np.float32)
    pos, box = W.uniform(n, box, 99)
    cfg = W.Config(pos=pos, box=box, rcut=np.array([[3.0]], np.float32), skin=0.4, name="gas")
    nbr, cnt, ovf = _paper_rows(cfg, {"leaf_size": 8, "qbits": 10})
    fp = _check(cfg, 10, nbr, cnt, ovf, 512)
    _, _, h = P.cell_boxes(pos, box, None, 1, 10)
    want = P.false_positive_mean(n / float(np.prod(box.astype(np.float64))), 3.4, h[0])
    assert abs(fp - want) <= 0.25 * want, (fp, want)


def test_paper_mode_two_types():
    cfg = W.colloid_solvent(n_total=3000, seed=7)
    nbr, cnt, ovf = _paper_rows(cfg, {"leaf_size": 8, "qbits": 10})
    _check(cfg, 10, nbr, cnt, ovf, 512)


def test_paper_mode_long_box_per_axis_bins():
    # ideal gas in a 10 x 10 x 40 box, 8-bit bins: the z bins are 4 times the x and
    # y bins, and the false positives follow the per-axis closed form
    n = 4000
    pos, box = W.uniform(n, [10.0, 10.0, 40.0], 4545)
    cfg = W.Config(pos=pos, box=box, rcut=np.array([[1.6]], np.float32), skin=0.4, name="long_gas")
    nbr, cnt, ovf = _paper_rows(cfg, {"leaf_size": 4, "qbits": 8})
    fp = _check(cfg, 8, nbr, cnt, ovf, 512)
    _, _, h = P.cell_boxes(pos, box, None, 1, 8)
    R = float(np.float32(1.6)) + float(np.float32(0.4))
    want = P.false_positive_mean(n / 4000.0, R, h[0])
    iso = P.false_positive_mean(n / 4000.0, R, h[0].max())
    print(f"[paper] long box: {fp:.3f} false positives per particle (per-axis closed form {want:.3f}, "
          f"one bin width on every axis {iso:.3f})", flush=True)
    assert abs(fp - want) <= 0.25 * want and fp < 0.7 * iso


@pytest.mark.parametrize("qbits", [10, 16])
def test_paper_mode_slab_60x60x240(qbits):
    # a liquid slab (0.8) in vapor (0.02) in the served stream's 60 x 60 x 240 box:
    # the root box is about 60 x 60 x 240, so the z bins are 4 times the x and y bins.
    # All rows are computed; 1500 sampled rows (half of them in the liquid) and the
    # 300 particles nearest the box faces are checked against the oracle bracket.
    cfg = W.slab(6.0, seed=4747)
    nbr, cnt, ovf = _paper_rows(cfg, {"leaf_size": 8, "qbits": qbits})
    rng = np.random.default_rng(qbits)
    z = cfg.pos[:, 2].astype(np.float64)
    liquid = np.nonzero(np.abs(z - 120.0) < 3.0)[0]
    face = np.min(np.minimum(cfg.pos, cfg.box - cfg.pos) / cfg.box, axis=1)
    q = np.unique(np.concatenate([rng.choice(liquid, 750, replace=False), rng.choice(cfg.n, 750, replace=False),
                                  np.argsort(face)[:300]]))
    fp = _check(cfg, qbits, nbr, cnt, ovf, 512, queries=q)
    ex = oracle.neighbor_counts(cfg.pos, cfg.box, cfg.rcut, cfg.skin)
    fp_all = float(cnt.sum() - ex.sum()) / cfg.n
    print(f"[paper] slab N={cfg.n} bits {qbits}: {fp:.3f} false positives per checked row, "
          f"{fp_all:.3f} per particle over all rows", flush=True)
    assert np.all(cnt >= ex)
