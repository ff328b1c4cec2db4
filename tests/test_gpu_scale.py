"""Parity at the full sizes of the Lennard-Jones workloads (N = 1M and 8M,
density 0.85, rc 3.0 + skin 0.4, max_nbr 256), of the 1M WCA fluid (short
cutoff) and of the 1M spinodal-like liquid-vapor configuration, in the launch
configuration the benchmark times: every count against the oracle's cell list,
and complete rows for a seeded sample of particles; at 1M, every row of
every single-system configuration."""
import numpy as np
import pytest

import oracle
import paper_1901_08088_amd as Q
import workloads as W

from nlist_check import require_gpu

pytestmark = pytest.mark.gpu

from bench import BENCH_OPTS  # the launch configuration bench.py times


@pytest.mark.parametrize("n,kind", [(1_000_000, "lj"), (8_000_000, "lj"), (1_000_000, "wca"),
                                    (1_000_000, "spinodal")])
def test_lj_fluid_full_size(n, kind):
    torch = require_gpu()
    cfg = {"lj": W.lj_fluid, "wca": W.wca_fluid, "spinodal": W.spinodal}[kind](n)
    n = cfg.n
    print(f"[scale] {kind} N={n} L={cfg.box[0]:.4f}", flush=True)
    pos = torch.from_numpy(cfg.pos).cuda()
    tree = Q.qbvh_build(pos, None, cfg.box, 1, BENCH_OPTS)
    max_nbr = 256
    nbr = torch.empty((n, max_nbr), dtype=torch.int32, device="cuda")
    cnt = torch.empty(n, dtype=torch.int32, device="cuda")
    ovf = torch.empty(1, dtype=torch.int32, device="cuda")
    Q.nlist_build(tree, cfg.rcut, cfg.skin, max_nbr, nbr, cnt, ovf)
    torch.cuda.synchronize()
    gcnt = cnt.cpu().numpy().astype(np.int64)
    ocnt = oracle.neighbor_counts(cfg.pos, cfg.box, cfg.rcut, cfg.skin)
    bad = np.nonzero(gcnt != ocnt)[0]
    assert bad.size == 0, f"{bad.size} count mismatches, first {bad[:5].tolist()}"
    assert int(ovf.item()) == int((ocnt > max_nbr).any())
    # complete rows for a sample, including the particles nearest the box faces
    rng = np.random.default_rng(n)
    face = np.argsort(np.min(np.minimum(cfg.pos, cfg.box - cfg.pos), axis=1))[:500]
    sample = np.unique(np.concatenate([rng.choice(n, 3000, replace=False), face]))
    rows = nbr[torch.from_numpy(sample).cuda()].cpu().numpy()
    rp, cols = oracle.neighbor_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, queries=sample)
    for q, i in enumerate(sample):
        c = gcnt[i]
        assert sorted(rows[q, :c].tolist()) == cols[rp[q]:rp[q + 1]].tolist(), i
    print(f"[scale] {kind} N={n} pairs={int(gcnt.sum())} mean={gcnt.mean():.3f} ok", flush=True)


@pytest.mark.parametrize("kind", ["lj", "colloid"])
def test_raw_rows_are_deterministic_at_1m(kind):
    # the same input built and listed twice: every raw row identical entry by
    # entry (not only as a set), every count and the flag identical
    torch = require_gpu()
    cfg = W.lj_fluid(1_000_000) if kind == "lj" else W.colloid_solvent(1_000_000)
    n = cfg.n
    print(f"[scale] determinism {kind} N={n}", flush=True)
    pos = torch.from_numpy(cfg.pos).cuda()
    types = None if cfg.types is None else torch.from_numpy(cfg.types).cuda()
    out = []
    for rep in range(2):
        tree = Q.qbvh_build(pos, types, cfg.box, cfg.ntypes, BENCH_OPTS)
        nbr = torch.full((n, 256), -7, dtype=torch.int32, device="cuda")
        cnt = torch.empty(n, dtype=torch.int32, device="cuda")
        ovf = torch.empty(1, dtype=torch.int32, device="cuda")
        Q.nlist_build(tree, cfg.rcut, cfg.skin, 256, nbr, cnt, ovf)
        torch.cuda.synchronize()
        out.append((nbr, cnt, int(ovf.item())))
        Q.qbvh_free(tree)
    assert torch.equal(out[0][1], out[1][1]) and out[0][2] == out[1][2]
    assert torch.equal(out[0][0], out[1][0])


@pytest.mark.timeout(600)
@pytest.mark.parametrize("kind", ["lj", "wca", "spinodal", "colloid"])
def test_every_row_at_1m(kind):
    # every row of the full-size 1M configurations against the oracle's cell
    # list, entry for entry as sets (rows sorted on both sides), in the launch
    # configuration the benchmark times
    torch = require_gpu()
    cfg = {"lj": W.lj_fluid, "wca": W.wca_fluid, "spinodal": W.spinodal,
           "colloid": W.colloid_solvent}[kind](1_000_000)
    n, max_nbr = cfg.n, 256
    print(f"[scale] every row {kind} N={n}", flush=True)
    pos = torch.from_numpy(cfg.pos).cuda()
    types = None if cfg.types is None else torch.from_numpy(cfg.types).cuda()
    tree = Q.qbvh_build(pos, types, cfg.box, cfg.ntypes, BENCH_OPTS)
    nbr = torch.empty((n, max_nbr), dtype=torch.int32, device="cuda")
    cnt = torch.empty(n, dtype=torch.int32, device="cuda")
    ovf = torch.empty(1, dtype=torch.int32, device="cuda")
    Q.nlist_build(tree, cfg.rcut, cfg.skin, max_nbr, nbr, cnt, ovf)
    torch.cuda.synchronize()
    gcnt = cnt.cpu().numpy().astype(np.int64)
    rp, cols = oracle.neighbor_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, types=cfg.types)
    ocnt = np.diff(rp)
    assert np.array_equal(gcnt, ocnt), f"{int(np.count_nonzero(gcnt != ocnt))} count mismatches"
    assert int(ovf.item()) == 0 and int(ocnt.max()) <= max_nbr
    g = nbr.cpu().numpy()
    del nbr
    listed = np.arange(max_nbr)[None, :] < gcnt[:, None]
    rows = np.repeat(np.arange(n, dtype=np.int64), gcnt)
    gkey = (rows << 32) | g[listed].astype(np.int64)
    del g, listed
    gkey.sort()
    okey = (rows << 32) | cols.astype(np.int64)
    assert np.array_equal(gkey, okey), f"{int(np.count_nonzero(gkey != okey))} entries differ"
    print(f"[scale] every row {kind} N={n}: {gkey.size} entries equal", flush=True)


@pytest.mark.parametrize("kind,radius", [("lj", 3.4), ("wca", 1.52)])
def test_cost_collapse_at_1m(kind, radius):
    # the cost model's build (costs carried up every level of the climb, then
    # the kept nodes marked) at a size with two upper levels: every count and
    # sampled rows against the oracle
    torch = require_gpu()
    cfg = W.lj_fluid(1_000_000) if kind == "lj" else W.wca_fluid(1_000_000)
    n = cfg.n
    opts = dict(BENCH_OPTS, collapse_radius=radius)
    print(f"[scale] cost collapse {kind} N={n} R={radius}", flush=True)
    pos = torch.from_numpy(cfg.pos).cuda()
    tree = Q.qbvh_build(pos, None, cfg.box, 1, opts)
    max_nbr = 256
    nbr = torch.empty((n, max_nbr), dtype=torch.int32, device="cuda")
    cnt = torch.empty(n, dtype=torch.int32, device="cuda")
    ovf = torch.empty(1, dtype=torch.int32, device="cuda")
    Q.nlist_build(tree, cfg.rcut, cfg.skin, max_nbr, nbr, cnt, ovf)
    torch.cuda.synchronize()
    gcnt = cnt.cpu().numpy().astype(np.int64)
    ocnt = oracle.neighbor_counts(cfg.pos, cfg.box, cfg.rcut, cfg.skin)
    assert np.array_equal(gcnt, ocnt), f"{int(np.count_nonzero(gcnt != ocnt))} count mismatches"
    assert int(ovf.item()) == int((ocnt > max_nbr).any())
    sample = np.sort(np.random.default_rng(n + 17).choice(n, 2000, replace=False))
    rows = nbr[torch.from_numpy(sample).cuda()].cpu().numpy()
    rp, cols = oracle.neighbor_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, queries=sample)
    for q, i in enumerate(sample):
        assert sorted(rows[q, :gcnt[i]].tolist()) == cols[rp[q]:rp[q + 1]].tolist(), i
    Q.qbvh_free(tree)
