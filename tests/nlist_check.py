"""Helpers shared by the GPU tests: run the HIP path through the C interface and
compare its output with the oracle."""
from __future__ import annotations

import numpy as np

import oracle
import paper_1901_08088_amd as Q


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a visible MI355X; run them with -m gpu on the GPU host")
    return torch


def to_dev(cfg):
    torch = require_gpu()
    pos = torch.from_numpy(np.ascontiguousarray(cfg.pos)).cuda()
    types = None if cfg.types is None else torch.from_numpy(np.ascontiguousarray(cfg.types)).cuda()
    return pos, types


def run_nlist(cfg, max_nbr=256, opts=None, tree=None, fill=-7):
    """qbvh_build + nlist_build on the GPU; returns (tree, nbr, count, overflow) on the host."""
    torch = require_gpu()
    pos, types = to_dev(cfg)
    tree = Q.qbvh_build(pos, types, cfg.box, cfg.ntypes, opts, tree=tree)
    n = cfg.n
    nbr = torch.full((max(n, 1), max(max_nbr, 1)), fill, dtype=torch.int32, device="cuda")
    cnt = torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda")
    ovf = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    Q.nlist_build(tree, cfg.rcut, cfg.skin, max_nbr, nbr if max_nbr > 0 else None, cnt, ovf)
    torch.cuda.synchronize()
    return tree, nbr.cpu().numpy()[:n, :max_nbr], cnt.cpu().numpy()[:n], int(ovf.item())


def compare_rows(cfg, nbr, cnt, ovf, max_nbr, queries=None, method="auto"):
    """Bit-exact comparison with the oracle.

    counts: equal for every compared row.  Rows with count <= max_nbr: the
    sorted stored entries equal the oracle row.  Overflowing rows: the stored
    max_nbr entries are distinct members of the oracle row.  Returns the
    oracle's (row_ptr, cols) for further checks.
    """
    rp, cols = oracle.neighbor_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, types=cfg.types,
                                     queries=queries, method=method)
    rows = np.arange(cfg.n) if queries is None else np.asarray(queries)
    ocnt = np.diff(rp)
    gcnt = cnt[rows].astype(np.int64)
    bad = np.nonzero(gcnt != ocnt)[0]
    assert bad.size == 0, (f"{bad.size} count mismatches, first rows {rows[bad[:5]].tolist()}: "
                           f"gpu {gcnt[bad[:5]].tolist()} oracle {ocnt[bad[:5]].tolist()}")
    if queries is None:
        assert ovf == int((ocnt > max_nbr).any())
    if max_nbr == 0:
        return rp, cols
    g = nbr[rows].astype(np.int64)
    stored = np.minimum(gcnt, max_nbr)
    col = np.arange(max_nbr)[None, :]
    big = np.iinfo(np.int64).max
    g = np.where(col < stored[:, None], g, big)
    g.sort(axis=1)
    ok_rows = ocnt <= max_nbr
    # expected: oracle rows padded with `big`
    exp = np.full((rows.size, max_nbr), big, dtype=np.int64)
    r_of = np.repeat(np.arange(rows.size), ocnt)
    within = np.arange(cols.size) - rp[r_of]
    sel = within < max_nbr
    exp[r_of[sel], within[sel]] = cols[sel]
    mism = np.nonzero(ok_rows & np.any(g != exp, axis=1))[0]
    assert mism.size == 0, f"{mism.size} row mismatches, first rows {rows[mism[:5]].tolist()}"
    for q in np.nonzero(~ok_rows)[0][:200]:
        row = set(cols[rp[q]:rp[q + 1]].tolist())
        got = g[q, :max_nbr]
        assert len(set(got.tolist())) == max_nbr and set(got.tolist()) <= row
    return rp, cols


def export(tree, what, n, dtype, width=1):
    torch = require_gpu()
    t = torch.empty((max(n, 1), width) if width > 1 else (max(n, 1),), dtype=dtype, device="cuda")
    Q.qbvh_export(tree, what, t)
    torch.cuda.synchronize()
    a = t.cpu().numpy()
    return a[:n]


def batch_buffers(cfgs, max_nbr=256, fill=-7):
    """Device inputs and fresh output buffers for nlist_build_many, one dict per system."""
    torch = require_gpu()
    systems = []
    for c in cfgs:
        pos, types = to_dev(c)
        n = c.n
        systems.append(dict(pos=pos, types=types, ntypes=c.ntypes, box=c.box, rcut=c.rcut, skin=c.skin,
                            max_nbr=max_nbr,
                            nbr=torch.full((max(n, 1), max(max_nbr, 1)), fill, dtype=torch.int32, device="cuda"),
                            count=torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda"),
                            overflow=torch.full((1,), -1, dtype=torch.int32, device="cuda")))
    return systems


def batch_results(systems, cfgs, rows=None):
    """Host copies (nbr, count, overflow) of every system; ``rows`` limits the copied rows."""
    torch = require_gpu()
    torch.cuda.synchronize()
    out = []
    for s, c in zip(systems, cfgs):
        n, m = c.n, s["max_nbr"]
        cnt = s["count"].cpu().numpy()[:n]
        if rows is None:
            nbr = s["nbr"].cpu().numpy()[:n, :m]
        else:
            idx = torch.as_tensor(np.asarray(rows[c.name] if isinstance(rows, dict) else rows), device="cuda")
            nbr = s["nbr"].index_select(0, idx.long()).cpu().numpy()[:, :m]
        out.append((nbr, cnt, int(s["overflow"].item())))
    return out
