"""Batched form: nlist_build_many over many independent systems of uneven size,
checked system by system against the oracle and against the single-system
path (identical counts), eager and graph-replayed, while tuning and after."""
import numpy as np
import pytest

import oracle

import paper_1901_08088_amd as Q
import workloads as W

from nlist_check import batch_buffers, batch_results, compare_rows, require_gpu, run_nlist

pytestmark = pytest.mark.gpu


def _mixed_systems():
    cfgs = [W.lj_fluid(4000)]
    cfgs += W.ensemble(6, n_min=800, n_max=30_000, scale=1.0)
    cfgs.append(W.colloid_solvent(n_total=3000, seed=7))
    one = W.Config(pos=np.array([[1.0, 2.0, 3.0]], dtype=np.float32), box=np.full(3, 10.0, np.float32),
                   rcut=np.array([[3.0]], np.float32), skin=0.4, name="single")
    empty = W.Config(pos=np.zeros((0, 3), np.float32), box=np.full(3, 10.0, np.float32),
                     rcut=np.array([[3.0]], np.float32), skin=0.4, name="empty")
    empty2 = W.Config(pos=np.zeros((0, 3), np.float32), box=np.full(3, 10.0, np.float32),
                      rcut=np.array([[1.0, 2.0], [2.0, 3.0]], np.float32), skin=0.4,
                      types=np.zeros(0, np.int32), name="empty, two types")
    cfgs += [one, empty, empty2, _four_types(37, seed=3)]
    return cfgs


def _four_types(n, seed):
    """Small four-type system: uneven type sizes, one type empty, two of equal size."""
    pos, box = W.uniform(n, [12.0, 12.0, 12.0], seed=seed)
    k = np.arange(n)
    types = np.where(k % 9 == 0, 3, np.where(k % 9 == 1, 1, 0)).astype(np.int32)  # type 2 empty
    if n >= 4:
        types[-2:] = 1  # ties between counts become likely for small n
    rcut = np.array([[1.5, 2.0, 1.0, 2.5], [2.0, 1.0, 0.0, 1.5], [1.0, 0.0, 2.0, 1.0], [2.5, 1.5, 1.0, 2.2]],
                    np.float32)
    return W.Config(pos=pos, box=box, rcut=rcut, skin=0.3, types=types, name=f"four types N={n}")


def _check_all(cfgs, res, max_nbr, plain_counts=None):
    for k, (c, (nbr, cnt, ovf)) in enumerate(zip(cfgs, res)):
        print(f"[batch] system {k} {c.name} N={c.n}", flush=True)
        if c.n == 0:
            assert ovf == 0
            continue
        compare_rows(c, nbr, cnt, ovf, max_nbr)
        if plain_counts is not None:
            assert np.array_equal(cnt, plain_counts[k]), f"system {k}: counts differ from the single-system path"


def _plain_counts(cfgs, max_nbr):
    out = []
    for c in cfgs:
        if c.n == 0:
            out.append(np.zeros(0, np.int32))
            continue
        tree, _, cnt, _ = run_nlist(c, max_nbr=max_nbr)
        Q.qbvh_free(tree)
        out.append(cnt)
    return out


@pytest.mark.parametrize("opts", [dict(leaf_size=4, qbits=16, block_size=128, eager=1),
                                  dict(leaf_size=1, qbits=10, block_size=64, eager=0),
                                  dict(leaf_size=8, qbits=12, block_size=256, eager=0),
                                  dict(leaf_size=16, qbits=16, block_size=64, eager=0)])
def test_batch_matches_oracle_and_plain(opts):
    require_gpu()
    cfgs = _mixed_systems()
    systems = batch_buffers(cfgs, max_nbr=256)
    print(f"[batch] opts {opts}", flush=True)
    Q.nlist_build_many(systems, opts)
    _check_all(cfgs, batch_results(systems, cfgs), 256, _plain_counts(cfgs, 256))


@pytest.mark.parametrize("sizes", [(1,), (1, 0), (0, 2), (2, 1)])
def test_batch_tiny_totals(sizes):
    """Batches whose concatenation holds one or two particles: the sort then
    runs on an array of one or two elements and must still give every
    position its value."""
    require_gpu()
    cfgs = []
    for k, n in enumerate(sizes):
        pos = np.array([[1.0, 2.0, 3.0], [1.5, 2.5, 3.0]], np.float32)[:n]
        cfgs.append(W.Config(pos=pos.reshape(-1, 3), box=np.full(3, 8.0, np.float32), rcut=np.array([[2.0]], np.float32),
                             skin=0.3, name=f"tiny {k} N={n}"))
    systems = batch_buffers(cfgs, max_nbr=8)
    print(f"[batch] tiny totals {sizes}", flush=True)
    Q.nlist_build_many(systems, dict(leaf_size=4))
    _check_all(cfgs, batch_results(systems, cfgs), 8)


def test_batch_overflow_and_scalar_rows():
    """max_nbr = 37: rows take scalar stores, many rows overflow."""
    require_gpu()
    cfgs = _mixed_systems()
    systems = batch_buffers(cfgs, max_nbr=37)
    Q.nlist_build_many(systems, dict(leaf_size=4, block_size=192))
    res = batch_results(systems, cfgs)
    assert any(r[2] == 1 for r in res)
    _check_all(cfgs, res, 37)


def test_batch_graph_replays_follow_new_inputs():
    """One shape, new positions every call: every replay of the captured graph
    matches the oracle for that call's inputs, with eager work and host syncs
    between the replays."""
    torch = require_gpu()
    base = W.ensemble(5, n_min=1500, n_max=20_000)
    opts = dict(leaf_size=4, qbits=16, block_size=128)
    for rep in range(3):
        cfgs = []
        for c in base:
            pos, box = W.lj_lattice(c.n, c.meta["rho"], 1000 + rep * 17 + c.meta["index"])
            cfgs.append(W.Config(pos=pos, box=box, rcut=c.rcut, skin=c.skin, name=c.name, meta=c.meta))
        systems = batch_buffers(cfgs, max_nbr=256)
        print(f"[batch] replay {rep}", flush=True)
        Q.nlist_build_many(systems, opts)
        junk = torch.randn(1 << 20, device="cuda")
        torch.cuda.synchronize()
        assert float(junk.abs().sum()) > 0
        _check_all(cfgs, batch_results(systems, cfgs), 256)
    st = Q.nlist_batch_stats()
    assert st["graphs_captured"] == 1 and st["tuned"] == 1


def test_batch_autotuner_freezes_and_stays_exact():
    require_gpu()
    cfgs = W.ensemble(8, n_min=2000, n_max=40_000)
    systems = batch_buffers(cfgs, max_nbr=256)
    calls = 0
    while True:
        Q.nlist_build_many(systems)
        calls += 1
        st = Q.nlist_batch_stats()
        if st["tuned"]:
            break
        assert calls <= 2 * st["candidates"] + 8, st
    print(f"[batch] tuned after {calls} calls: {st}", flush=True)
    assert st["leaf_size"] in (4, 8, 16) and st["qbits"] in (10, 16) and st["block_size"] in (64, 128, 256)
    for s in systems:
        s["count"].fill_(-1)
        s["nbr"].fill_(-7)
    Q.nlist_build_many(systems)
    _check_all(cfgs, batch_results(systems, cfgs), 256, _plain_counts(cfgs, 256))


@pytest.mark.timeout(900)
def test_batch_full_ensemble():
    """The 256-replica ensemble at full size (N log-uniform in [2000, 200000],
    density 0.3-0.9, rc 2.5-3.0, skin 0.4, max_nbr 256), graph-replayed after
    tuning: every count of every replica equals the oracle's (and the
    single-system path's), sampled rows of every replica and every row of
    every eighth replica equal the oracle's."""
    torch = require_gpu()
    cfgs = W.ensemble()
    total = sum(c.n for c in cfgs)
    print(f"[batch] 256 replicas, {total:,} particles", flush=True)
    systems = batch_buffers(cfgs, max_nbr=256)
    for _ in range(60):
        Q.nlist_build_many(systems)
        if Q.nlist_batch_stats()["tuned"]:
            break
    Q.nlist_build_many(systems)
    rng = np.random.default_rng(5)
    rows = {c.name: np.sort(rng.choice(c.n, min(12, c.n), replace=False)) for c in cfgs}
    res = batch_results(systems, cfgs, rows=rows)
    plain = _plain_counts(cfgs, 256)
    checked = 0
    for k, c in enumerate(cfgs):
        nbr, cnt, ovf = res[k]
        ocnt = oracle.neighbor_counts(c.pos, c.box, c.rcut, c.skin, method="cells")
        assert np.array_equal(cnt.astype(np.int64), ocnt), f"replica {k}: counts differ from the oracle"
        if k % 32 == 31:
            print(f"[batch] replicas 0..{k}: counts equal to the oracle's", flush=True)
        assert ovf == int((ocnt > 256).any())
        assert np.array_equal(cnt, plain[k]), f"replica {k}: counts differ from the single-system path"
        q = rows[c.name]
        full = np.full((c.n, 256), -7, np.int32)
        full[q] = nbr
        compare_rows(c, full, cnt, ovf, 256, queries=q, method="cells")
        if k % 8 == 0:
            # every row of every eighth replica
            compare_rows(c, systems[k]["nbr"].cpu().numpy()[:c.n, :256], cnt, ovf, 256, method="cells")
            checked += c.n
    print(f"[batch] every row of 32 replicas ({checked:,} particles) equal to the oracle's", flush=True)
    print(f"[batch] stats {Q.nlist_batch_stats()}", flush=True)
    del systems
    torch.cuda.empty_cache()
