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


def _check(cfg, qbits, nbr, cnt, ovf, max_nbr):
    assert ovf == 0 and cnt.max() <= max_nbr
    lo_rp, lo_c = P.paper_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, types=cfg.types, qbits=qbits)
    hi_rp, hi_c = P.paper_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, types=cfg.types, qbits=qbits, pad=0.05)
    ex_rp, ex_c = oracle.neighbor_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, types=cfg.types)
    for i in range(cfg.n):
        row = nbr[i, :cnt[i]]
        got = set(row.tolist())
        assert len(got) == cnt[i], f"row {i} has duplicates"
        assert set(lo_c[lo_rp[i]:lo_rp[i + 1]].tolist()) <= got, f"row {i} misses a paper-mode neighbor"
        assert got <= set(hi_c[hi_rp[i]:hi_rp[i + 1]].tolist()), f"row {i} lists a particle beyond the pad"
        assert set(ex_c[ex_rp[i]:ex_rp[i + 1]].tolist()) <= got
    return float(cnt.sum() - (ex_rp[-1])) / cfg.n


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
    want = P.false_positive_mean(n / float(np.prod(box.astype(np.float64))), 3.4, float(h[0]))
    assert abs(fp - want) <= 0.25 * want, (fp, want)


def test_paper_mode_two_types():
    cfg = W.colloid_solvent(n_total=3000, seed=7)
    nbr, cnt, ovf = _paper_rows(cfg, {"leaf_size": 8, "qbits": 10})
    _check(cfg, 10, nbr, cnt, ovf, 512)
