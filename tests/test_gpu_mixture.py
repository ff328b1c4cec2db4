"""The binary colloid-solvent mixture: two particle types, one tree per type,
per-type-pair cutoffs rc_ij = (sigma_i + sigma_j) / 2 + skin 0.4 (solvent
sigma 1, colloid sigma 5, 2% colloids by number, random sequential addition
with no overlaps)."""
import numpy as np
import pytest

import oracle

import paper_1901_08088_amd as Q
import workloads as W

from nlist_check import compare_rows, require_gpu, run_nlist

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("opts", [None, {"leaf_size": 8, "block_size": 256}])
def test_mixture_100k_rows(opts):
    require_gpu()
    cfg = W.colloid_solvent(100_000)
    print(f"[mixture] N={cfg.n} L={cfg.box[0]:.3f} opts={opts}", flush=True)
    tree, nbr, cnt, ovf = run_nlist(cfg, max_nbr=256, opts=opts)
    info = Q.qbvh_info(tree)
    assert info["ntypes"] == 2
    assert list(info["tree_count"][:2]) == [int((cfg.types == 0).sum()), int((cfg.types == 1).sum())]
    compare_rows(cfg, nbr, cnt, ovf, 256, method="cells")
    Q.qbvh_free(tree)


@pytest.mark.timeout(900)
def test_mixture_1m_sampled():
    """Full size (1,000,000 particles), in the benchmark's launch
    configuration: every count equal to the oracle's, and the rows of a
    20,000-row sample plus all colloids exact."""
    require_gpu()
    from bench import BENCH_OPTS
    cfg = W.colloid_solvent(1_000_000)
    print(f"[mixture] N={cfg.n} L={cfg.box[0]:.3f} colloids={cfg.meta['n_colloid']}", flush=True)
    tree, nbr, cnt, ovf = run_nlist(cfg, max_nbr=256, opts=BENCH_OPTS)
    ocnt = oracle.neighbor_counts(cfg.pos, cfg.box, cfg.rcut, cfg.skin, types=cfg.types, method="cells")
    bad = np.nonzero(cnt.astype(np.int64) != ocnt)[0]
    assert bad.size == 0, f"{bad.size} counts differ from the oracle, first rows {bad[:5].tolist()}"
    assert ovf == int((ocnt > 256).any())
    rng = np.random.default_rng(9)
    q = np.union1d(rng.choice(cfg.n, 20_000, replace=False), np.nonzero(cfg.types == 1)[0])
    compare_rows(cfg, nbr, cnt, ovf, 256, queries=q, method="cells")
    Q.qbvh_free(tree)
