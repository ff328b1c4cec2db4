#!/usr/bin/env python3
"""Benchmark: exact neighbor-list builds per second on one MI355X.

One step = the whole hot path on one synthetic configuration: qbvh_build
(Morton codes, radix sort, gather, radix tree, bottom-up boxes, quantized
preorder layout) followed by nlist_build (stackless traversal with the exact
distance filter, rows written to a device [N][max_nbr] buffer).  Inputs are
resident in device memory before the timed region.

Default workload: Lennard-Jones fluid stand-in, N = 8,000,000, density 0.85,
rc = 3.0 + skin 0.4, max_nbr = 256, fp32 coordinates (jittered simple-cubic
lattice, seeded).

Prints one JSON line (see the field list at the bottom of ``main``).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

import hashlib  # noqa: E402
import re  # noqa: E402

METRIC = "nlist builds/s & pairs/s at 1 GPU vs oracle; batched vs plain; HBM GB/s %"
HBM_PEAK_GBS = 8000.0
BENCH_OPTS = {"leaf_size": 16, "qbits": 16, "block_size": 64}
WORKLOADS = {
    "lj8m": dict(n=8_000_000, rho=0.85, rc=3.0, skin=0.4, max_nbr=256),
    "lj1m": dict(n=1_000_000, rho=0.85, rc=3.0, skin=0.4, max_nbr=256),
    "lj4000": dict(n=4000, rho=0.85, rc=3.0, skin=0.4, max_nbr=256),
    # two-type colloid/solvent mixture (one tree per type), 2% colloids of diameter 5
    "colloid1m": dict(n=1_000_000, kind="colloid", skin=0.4, max_nbr=256),
    # WCA short cutoff (rc = 2^(1/6)) and a spinodal-like liquid (0.75) / vapor (0.05) structure
    "wca1m": dict(n=1_000_000, kind="wca", rho=0.85, skin=0.4, max_nbr=64),
    "spinodal1m": dict(n=1_000_000, kind="spinodal", skin=0.4, max_nbr=256),
}


def make_config(wl: dict):
    if wl.get("kind") == "colloid":
        return W.colloid_solvent(wl["n"], skin=wl["skin"])
    if wl.get("kind") == "wca":
        return W.wca_fluid(wl["n"], rho=wl["rho"], skin=wl["skin"])
    if wl.get("kind") == "spinodal":
        return W.spinodal(wl["n"], skin=wl["skin"])
    return W.lj_fluid(wl["n"], rho=wl["rho"], rc=wl["rc"], skin=wl["skin"])


def describe(wl: dict, cfg) -> str:
    if wl.get("kind") == "colloid":
        m = cfg.meta
        return (f"colloid_solvent N={cfg.n:,} ({m['n_colloid']:,} colloids d=5, {m['n_solvent']:,} solvent, "
                f"L={m['L']:.2f}, colloid volume fraction {m['colloid_volume_fraction']:.3f}) rc_ij=(d_i+d_j)/2 "
                f"skin={wl['skin']} max_nbr={wl['max_nbr']} fp32, one tree per type (RSA placement, seed "
                f"{m['seed']})")
    if wl.get("kind") == "wca":
        return (f"wca_fluid N={cfg.n:,} rho={wl['rho']} rc=2^(1/6) skin={wl['skin']} max_nbr={wl['max_nbr']} "
                f"fp32 (jittered simple-cubic lattice, seed {cfg.meta['seed']})")
    if wl.get("kind") == "spinodal":
        m = cfg.meta
        return (f"spinodal N={cfg.n:,} (liquid 0.75 / vapor 0.05 bicontinuous domains of {m['wavelength']:g} sigma, "
                f"L={m['L']:.2f}) rc=3.0 skin={wl['skin']} max_nbr={wl['max_nbr']} fp32 (seed {m['seed']})")
    return (f"lj_fluid N={cfg.n:,} rho={wl['rho']} rc={wl['rc']} skin={wl['skin']} "
            f"max_nbr={wl['max_nbr']} fp32 (jittered simple-cubic lattice, seed {cfg.meta['seed']})")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def traversal_bytes(n: int, nrecords: int, stored_pairs: int) -> int:
    """Algorithmic HBM bytes of one traversal launch: the Z-ordered particle
    array (16 B per particle, queries and candidates alike) read once, every
    record (32 B) and its rope (4 B) read once, every stored neighbor index
    (4 B) and every count (4 B) written once."""
    return 16 * n + 36 * nrecords + 4 * stored_pairs + 4 * n


def host_info() -> dict:
    """CPU model and core counts of the host the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo", encoding="utf-8") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    import oracle
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
            "oracle_threads": oracle.max_threads()}


def gpu_rows(nbr, rows):
    """Host copy of the GPU rows ``rows`` of the device list ``nbr``."""
    import torch
    idx = torch.as_tensor(np.asarray(rows, dtype=np.int64), device=nbr.device)
    return nbr.index_select(0, idx).cpu().numpy()


def row_parity(cfg, g_nbr_rows, g_cnt, max_nbr, queries, rp, cols):
    """Compare GPU rows with the oracle's on ``queries`` (rows not overflowing):
    entries in one row and not the other, split into band pairs (|d - r_list|
    within 1e-5 r_list, where another rounding order may decide differently)
    and mismatches (everything else)."""
    import oracle
    queries = np.asarray(queries)
    c = g_cnt[queries].astype(np.int64)
    ok = c <= max_nbr
    big = np.iinfo(np.int64).max
    col = np.arange(max_nbr)[None, :]
    g = np.where(col < c[:, None], g_nbr_rows.astype(np.int64), big)
    g.sort(axis=1)
    ocnt = np.diff(rp)
    exp = np.full((queries.size, max_nbr), big, dtype=np.int64)
    r_of = np.repeat(np.arange(queries.size), ocnt)
    within = np.arange(cols.size) - rp[r_of]
    sel = within < max_nbr
    exp[r_of[sel], within[sel]] = cols[sel]
    differ = np.nonzero(ok & ((ocnt != c) | np.any(g != exp, axis=1)))[0]
    L = np.asarray(cfg.box, dtype=np.float64)
    pos = cfg.pos.astype(np.float64)
    r2 = oracle.rlist2_table(cfg.rcut, cfg.skin)
    t = np.zeros(cfg.n, np.int64) if cfg.types is None else cfg.types.astype(np.int64)
    band = mism = 0
    for k in differ:
        i = int(queries[k])
        got = g[k][g[k] != big]
        for j in np.setxor1d(got, cols[rp[k]:rp[k + 1]]):
            d = pos[j] - pos[i]
            s = d / L
            d = d - L * np.trunc(s + np.copysign(0.5, s))  # nearest image, halves away from zero
            dist = np.sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2])
            r = np.sqrt(max(r2[t[i], t[j]], 0.0))
            if abs(dist - r) <= 1e-5 * r:
                band += 1
            else:
                mism += 1
    return {"rows_checked": int(np.count_nonzero(ok)), "band_pair_differences": band, "mismatches": mism}


def band_report(cfg, queries=None, threads: int = 0) -> dict:
    """Band pairs (directed) over the queried rows, both readings of the 1e-5 tolerance."""
    import oracle
    t0 = time.perf_counter()
    a, b = oracle.band_counts(cfg.pos, cfg.box, cfg.rcut, cfg.skin, types=cfg.types, queries=queries,
                              nthreads=threads)
    return {"rows": int(cfg.n if queries is None else len(queries)), "rel_1e-5": int(a.sum()),
            "abs_1e-5_sigma": int(b.sum()), "seconds": time.perf_counter() - t0}


# HBM traffic of one k_traverse launch on lj8m with BENCH_OPTS, from two rocprofv3
# counter passes (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) divided by the
# factor the same counters read for a plain elementwise copy of known size (the
# --copy-probe-mib kernel).  Valid only for the kernel sources it was taken on:
# ``traffic`` is reported as null once their hash differs.
TRAFFIC = {"sources": "46520ba402bbbee4", "workload": "lj8m",
           "opts": {"leaf_size": 16, "qbits": 16, "block_size": 64},
           "fetch_kib": 1528910.0, "write_kib": 6610126.0, "copy_factor": 1.0,
           # FETCH_SIZE per byte read: 0.500 for vector loads (the copy probe), 1.000 for
           # scalar loads (profiles/fetch_size_calibration.md)
           "fetch_factor": 0.500012, "fetch_factor_scalar": 1.000049,
           "profile": "profiles/k_traverse_lj8m_counters.md",
           # SQ_INSTS_VALU x 4 / (1024 SIMDs x kernel cycles): the VALU issues one wave64
           # instruction per 4 cycles per SIMD, so this is the kernel's VALU issue roofline
           "valu_busy": 0.90}
KERNEL_SOURCES = ("paper_1901_08088_amd/csrc/traverse.hip", "paper_1901_08088_amd/csrc/qbvh_internal.h",
                  "paper_1901_08088_amd/csrc/build_common.h", "paper_1901_08088_amd/csrc/launch_geometry.h")


def _code_only(text: str) -> str:
    """The source with comments and blank space removed: a comment edit does not
    change the kernel the counters were taken on.  (No string literal in these
    sources holds a comment marker.)"""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, opts: dict, scalar_reads: bool = False):
    """HBM bytes per traversal launch from the committed counter summary, or None
    when the kernel sources, workload or options differ from the profiled ones.
    Each counter is scaled by what it reads for the copy probe (FETCH_SIZE counts
    half of the bytes read by vector loads, WRITE_SIZE all bytes written);
    scalar_reads: scale FETCH_SIZE as for scalar loads instead (which it counts
    in full), the lower end of the range."""
    t = TRAFFIC
    if t is None or t["sources"] != kernel_source_hash() or t["workload"] != workload or t["opts"] != opts:
        return None
    ff = t["fetch_factor_scalar"] if scalar_reads else t["fetch_factor"]
    return (t["fetch_kib"] / ff + t["write_kib"] / t["copy_factor"]) * 1024.0


def copy_probe(mib: int) -> None:
    """One plain elementwise kernel (negation) reading and writing ``mib`` MiB,
    launched three times after the timed region: the reference a counter pass
    uses to scale FETCH_SIZE / WRITE_SIZE to bytes."""
    import torch
    src = torch.ones(mib * (1 << 18), dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    log(f"copy probe: {mib} MiB read + {mib} MiB written per launch, 3 launches")


def paper_mode(cfg, pos, steps: int) -> dict:
    """Exact vs paper-mode lists (Section 2.3: leaf-box overlap, no distance
    check) on the same workload with the paper's 10-bit grid: traversal time
    of each and the paper mode's extra entries per particle."""
    import torch
    import paper_1901_08088_amd as Q
    opts = dict(BENCH_OPTS, qbits=10)
    tree = Q.qbvh_build(pos, None, cfg.box, 1, opts)
    n = cfg.n
    nbr = torch.empty((n, 320), dtype=torch.int32, device="cuda")
    cnt = torch.empty(n, dtype=torch.int32, device="cuda")
    ovf = torch.empty(1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    out = {"workload": f"same configuration, 10-bit grid, leaf {opts['leaf_size']}, max_nbr 320"}
    for name, mode in (("exact", Q.LIST_EXACT), ("paper", Q.LIST_PAPER)):
        for _ in range(2):
            Q.nlist_build_ex(tree, cfg.rcut, cfg.skin, 320, mode, nbr, cnt, ovf)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(steps):
            Q.nlist_build_ex(tree, cfg.rcut, cfg.skin, 320, mode, nbr, cnt, ovf)
        ev[1].record(stream)
        torch.cuda.synchronize()
        out[f"{name}_traverse_ms"] = ev[0].elapsed_time(ev[1]) / steps
        out[f"{name}_pairs"] = int(cnt.sum())
        out[f"{name}_overflow"] = int(ovf.item())
    out["false_positives_per_particle"] = (out["paper_pairs"] - out["exact_pairs"]) / n
    Q.qbvh_free(tree)
    del nbr
    torch.cuda.empty_cache()
    log(f"paper mode: {out}")
    return out


def f64_data(cfg, max_nbr: int, steps: int) -> dict:
    """The same configuration as fp64 particle data (every coordinate moved by
    up to 1e-3 sigma in fp64, so it is not an fp32 value): qbvh_build_f64 +
    nlist_build timed like the main leg; lists exact for the fp64 data."""
    import torch
    import paper_1901_08088_amd as Q
    c64 = W.as_f64(cfg, seed=19010889)
    n = c64.n
    pos = torch.from_numpy(c64.pos).cuda()
    types = None if c64.types is None else torch.from_numpy(c64.types).cuda()
    nbr = torch.empty((n, max_nbr), dtype=torch.int32, device="cuda")
    cnt = torch.empty(n, dtype=torch.int32, device="cuda")
    ovf = torch.empty(1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    tree = Q.qbvh_build(pos, types, c64.box, c64.ntypes, BENCH_OPTS)
    for _ in range(2):
        Q.qbvh_build(pos, types, c64.box, c64.ntypes, BENCH_OPTS, tree=tree)
        Q.nlist_build(tree, c64.rcut, c64.skin, max_nbr, nbr, cnt, ovf)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    torch.cuda.synchronize()
    for e in ev:
        e[0].record(stream)
        Q.qbvh_build(pos, types, c64.box, c64.ntypes, BENCH_OPTS, tree=tree)
        e[1].record(stream)
        Q.nlist_build(tree, c64.rcut, c64.skin, max_nbr, nbr, cnt, ovf)
        e[2].record(stream)
    torch.cuda.synchronize()
    out = {"workload": "same configuration as fp64 data (offsets up to 1e-3 sigma, seed 19010889)",
           "build_ms": float(np.mean([e[0].elapsed_time(e[1]) for e in ev])),
           "traverse_ms": float(np.mean([e[1].elapsed_time(e[2]) for e in ev])),
           "directed_pairs": int(cnt.sum()), "overflow": int(ovf.item())}
    out["builds_per_s"] = 1e3 / (out["build_ms"] + out["traverse_ms"])
    Q.qbvh_free(tree)
    del nbr
    torch.cuda.empty_cache()
    log(f"fp64 data: {out}")
    return out


def grid_comparator(cfg, pos, max_nbr: int, steps: int) -> dict:
    """The same lists by the grid method the paper compares its tree with
    (nlist_build_grid: cells at least as wide as the list radius, particles
    sorted by cell, 27 cells per particle scanned by n cooperating lanes),
    timed over ``steps`` calls for every n in 1..32; the fastest n is the
    comparator (the paper reports the grid at its best n)."""
    import torch
    import paper_1901_08088_amd as Q
    n = cfg.n
    nbr = torch.empty((n, max_nbr), dtype=torch.int32, device="cuda")
    cnt = torch.empty(n, dtype=torch.int32, device="cuda")
    ovf = torch.empty(1, dtype=torch.int32, device="cuda")
    rc, skin = float(cfg.rcut[0, 0]), cfg.skin
    stream = torch.cuda.current_stream()
    g = None
    per = {}
    pairs = None
    for lanes in (1, 2, 4, 8, 16, 32):
        for _ in range(2):
            g = Q.nlist_build_grid(pos, cfg.box, rc, skin, max_nbr, nbr, cnt, ovf, grid=g, lanes=lanes)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(steps):
            Q.nlist_build_grid(pos, cfg.box, rc, skin, max_nbr, nbr, cnt, ovf, grid=g, lanes=lanes)
        ev[1].record(stream)
        torch.cuda.synchronize()
        per[lanes] = ev[0].elapsed_time(ev[1]) / steps
        p = int(cnt.sum())
        if pairs is not None and p != pairs:
            raise RuntimeError(f"grid pairs differ between lane counts: {p} != {pairs}")
        pairs = p
    best = min(per, key=per.get)
    out = {"method": "uniform grid, cells >= r_list, particles sorted by cell, 27-cell scan by n cooperating "
                     "lanes per particle (best n reported)",
           "ms": per[best], "lanes": best, "ms_per_lanes": {str(k): v for k, v in per.items()},
           "directed_pairs": pairs}
    g.free()
    del nbr
    torch.cuda.empty_cache()
    log(f"grid comparator: {out}")
    return out


def single_graph(cfg, pos, types, max_nbr: int, steps: int) -> dict:
    """The same system as a one-system nlist_build_many call with the bench's
    options fixed (no autotuning): build + traversal replayed from one captured
    hipGraph, against the same work launched kernel by kernel."""
    import torch
    import paper_1901_08088_amd as Q
    n = cfg.n
    y = dict(pos=pos, types=types, ntypes=cfg.ntypes, box=cfg.box, rcut=cfg.rcut, skin=cfg.skin,
             max_nbr=max_nbr, nbr=torch.empty((n, max_nbr), dtype=torch.int32, device="cuda"),
             count=torch.empty(n, dtype=torch.int32, device="cuda"),
             overflow=torch.empty(1, dtype=torch.int32, device="cuda"))
    stream = torch.cuda.current_stream()
    out = {}
    for name, eager in (("graph", 0), ("eager", 1)):
        o = dict(BENCH_OPTS, eager=eager)
        for _ in range(3):
            Q.nlist_build_many([y], o)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(steps):
            Q.nlist_build_many([y], o)
        ev[1].record(stream)
        torch.cuda.synchronize()
        out[f"{name}_ms"] = ev[0].elapsed_time(ev[1]) / steps
    out["pairs"] = int(y["count"].sum())
    out["graph_builds_per_s"] = 1e3 / out["graph_ms"]
    Q.nlist_batch_release()
    del y
    torch.cuda.empty_cache()
    log(f"one-system batched call: {out}")
    return out


def batched_vs_plain(steps: int) -> dict:
    """The 256-replica ensemble (N log-uniform in [2000, 200000], density
    0.3-0.9, rc 2.5-3.0, skin 0.4, max_nbr 256): one nlist_build_many call
    (autotuned, graph-replayed) against qbvh_build + nlist_build per replica
    in sequence on the same stream, both timed over ``steps`` passes."""
    import torch
    import paper_1901_08088_amd as Q
    cfgs = W.ensemble()
    total = sum(c.n for c in cfgs)
    log(f"ensemble: {len(cfgs)} replicas, {total:,} particles")
    systems = []
    for c in cfgs:
        systems.append(dict(pos=torch.from_numpy(c.pos).cuda(), types=None, ntypes=1, box=c.box, rcut=c.rcut,
                            skin=c.skin, max_nbr=256,
                            nbr=torch.empty((c.n, 256), dtype=torch.int32, device="cuda"),
                            count=torch.empty(c.n, dtype=torch.int32, device="cuda"),
                            overflow=torch.empty(1, dtype=torch.int32, device="cuda")))
    stream = torch.cuda.current_stream()
    trees = [None] * len(cfgs)

    def plain():
        for k, (c, y) in enumerate(zip(cfgs, systems)):
            trees[k] = Q.qbvh_build(y["pos"], None, c.box, 1, BENCH_OPTS, tree=trees[k])
            Q.nlist_build(trees[k], c.rcut, c.skin, 256, y["nbr"], y["count"], y["overflow"])

    def timed(fn):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(steps):
            fn()
        ev[1].record(stream)
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / steps

    for _ in range(3):
        plain()
    plain_ms = timed(plain)
    plain_pairs = int(sum(int(y["count"].sum()) for y in systems))
    log(f"plain: {plain_ms:.3f} ms per pass over all replicas")
    calls = 0
    while not Q.nlist_batch_stats()["tuned"] or calls < 2:
        Q.nlist_build_many(systems)
        calls += 1
        if calls > 200:
            raise RuntimeError("autotuner did not settle")
    torch.cuda.synchronize()
    st = Q.nlist_batch_stats()
    log(f"autotuner settled after {calls} calls: {st}")
    batch_ms = timed(lambda: Q.nlist_build_many(systems))
    batch_pairs = int(sum(int(y["count"].sum()) for y in systems))
    if batch_pairs != plain_pairs:
        raise RuntimeError(f"batched pairs {batch_pairs} != plain pairs {plain_pairs}")
    log(f"batched: {batch_ms:.3f} ms per call")
    # after timing: four replicas of the batched results (the smallest, the
    # largest and two drawn at random) against the oracle -- every count and
    # 500 sampled rows each
    import oracle
    rng = np.random.default_rng(3)
    sizes = [c.n for c in cfgs]
    picks = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), *rng.choice(len(cfgs), 2, replace=False).tolist()})
    checked = {}
    for k in picks:
        c, y = cfgs[k], systems[k]
        g_cnt = y["count"].cpu().numpy().astype(np.int64)
        o_cnt = oracle.neighbor_counts(c.pos, c.box, c.rcut, c.skin)
        q = np.sort(rng.choice(c.n, min(500, c.n), replace=False))
        rp, cols = oracle.neighbor_lists(c.pos, c.box, c.rcut, c.skin, queries=q)
        checked[c.name] = {"n": c.n, "count_mismatch_rows": int(np.count_nonzero(o_cnt != g_cnt)),
                           **row_parity(c, gpu_rows(y["nbr"], q), g_cnt, 256, q, rp, cols)}
    log(f"batched results checked: {checked}")
    for t in trees:
        Q.qbvh_free(t)
    Q.nlist_batch_release()
    return {"workload": f"256 LJ replicas, sum N = {total:,} (seed 19010885), rc 2.5-3.0 + skin 0.4, max_nbr 256",
            "systems": len(cfgs), "particles": total, "directed_pairs": batch_pairs,
            "plain_ms": plain_ms, "batched_ms": batch_ms,
            "plain_systems_per_s": len(cfgs) * 1e3 / plain_ms,
            "batched_systems_per_s": len(cfgs) * 1e3 / batch_ms,
            "batched_pairs_per_s": batch_pairs * 1e3 / batch_ms,
            "speedup": plain_ms / batch_ms, "plain_opts": BENCH_OPTS,
            "tuned": {k: st[k] for k in ("leaf_size", "qbits", "block_size", "candidates")},
            "tuning_calls": calls, "results_checked_after_timing": checked}


def served(seconds: float, load: float = 0.7) -> dict:
    """The served stream: 64 simulations (16 liquid-vapor slabs in 60 x 60 x 240
    boxes and 48 LJ fluids, N log-uniform in [1e4, 2e6], rc 3.0 + skin 0.4,
    max_nbr 256).  Each request is the simulation's previous positions plus a
    N(0, 0.05) displacement, wrapped, for a simulation drawn uniformly.  First
    the saturated throughput of the continuous-batching server is measured
    (a burst of 2 requests per simulation), then Poisson arrivals at ``load``
    times that rate run for ``seconds``, against the same stream served one
    request at a time in FIFO order (one stream, batches of one)."""
    import torch
    import paper_1901_08088_amd as Q
    sims = W.served_sims()
    total = sum(c.n for c in sims)
    log(f"served stream: {len(sims)} simulations, {total:,} particles")
    cur = [torch.from_numpy(c.pos).cuda() for c in sims]
    boxes = [torch.tensor(c.box, device="cuda") for c in sims]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(19010886)

    def move(k):
        p = cur[k] + 0.05 * torch.randn(cur[k].shape, device="cuda", generator=gen)
        p = torch.remainder(p, boxes[k])
        p = torch.where(p >= boxes[k], torch.zeros_like(p), p)
        cur[k] = p
        return p

    budget = 96 << 30

    def burst(srv, per_sim):
        order = [k for _ in range(per_sim) for k in range(len(sims))]
        t0 = time.perf_counter()
        ts = []
        for k in order:
            p = move(k)
            torch.cuda.current_stream().synchronize()
            ts.append(srv.submit(k, p, sims[k].box, sims[k].rcut, sims[k].skin, 256))
        for t in ts:
            srv.wait(t)
        return len(order) / (time.perf_counter() - t0)

    def poisson(srv, rate):
        rng = np.random.default_rng(11)
        t0 = time.perf_counter()
        nxt = t0
        ts = []
        while nxt - t0 < seconds:
            now = time.perf_counter()
            if nxt > now:
                time.sleep(max(0.0, nxt - now - 2e-4))
                while time.perf_counter() < nxt:
                    pass
            k = int(rng.integers(len(sims)))
            p = move(k)
            torch.cuda.current_stream().synchronize()
            ts.append(srv.submit(k, p, sims[k].box, sims[k].rcut, sims[k].skin, 256))
            nxt += rng.exponential(1.0 / rate)
            if len(ts) % 64 == 0:
                log(f"  {len(ts)} requests submitted")
        for t in ts:
            srv.wait(t)
        return srv.stats()

    out = {"workload": f"64 simulations (16 slabs 60x60x240 + 48 LJ fluids, N log-uniform 1e4-2e6, "
                       f"sum N = {total:,}, seed 19010886), rc 3.0 + skin 0.4, max_nbr 256",
           "seconds": seconds, "load": load}
    srv = Q.Server(budget, max_inflight=2, max_batch=64)
    burst(srv, 1)  # warm-up: sessions allocated, batch workspaces sized
    sat = burst(srv, 2)
    srv.close()
    rate = load * sat
    log(f"saturated: {sat:.1f} requests/s; Poisson arrivals at {rate:.1f}/s for {seconds:g} s")
    srv = Q.Server(budget, max_inflight=2, max_batch=64)
    burst(srv, 1)
    st = poisson(srv, rate)
    # after timing: the published results of four simulations (the smallest and
    # largest slab and LJ fluid) against the oracle on the positions of their
    # last request -- every count and 500 sampled rows each
    import oracle
    checked = {}
    picks = {min((c for c in sims if kind in c.name), key=lambda c: c.n).meta["sim"] for kind in ("slab", "_lj_")}
    picks |= {max((c for c in sims if kind in c.name), key=lambda c: c.n).meta["sim"] for kind in ("slab", "_lj_")}
    for k in sorted(picks):
        c = sims[k]
        moved = W.Config(pos=cur[k].cpu().numpy(), box=c.box, rcut=c.rcut, skin=c.skin, name=c.name)
        g_nbr, g_cnt, g_ovf = srv.read(k)
        o_cnt = oracle.neighbor_counts(moved.pos, moved.box, moved.rcut, moved.skin)
        q = np.sort(np.random.default_rng(k).choice(c.n, min(500, c.n), replace=False))
        rp, cols = oracle.neighbor_lists(moved.pos, moved.box, moved.rcut, moved.skin, queries=q)
        r = row_parity(moved, g_nbr[q], g_cnt.astype(np.int64), 256, q, rp, cols)
        checked[c.name] = {"n": c.n, "count_mismatch_rows": int(np.count_nonzero(o_cnt != g_cnt)),
                           "overflow": g_ovf, **r}
    srv.close()
    log(f"continuous batching: {st}; results checked: {checked}")
    fifo = Q.Server(budget, max_inflight=1, max_batch=1)
    burst(fifo, 1)
    fsat = burst(fifo, 1)
    fst = poisson(fifo, rate)
    fifo.close()
    log(f"one at a time: {fst}")
    keys = ("p50_ms", "p99_ms", "mean_ms", "requests_per_s", "particles_per_s", "mean_batch", "completed")
    out.update({"saturated_requests_per_s": sat, "arrival_rate_per_s": rate,
                "continuous_batching": {k: st[k] for k in keys},
                "results_checked_after_timing": checked,
                "fifo_saturated_requests_per_s": fsat,
                "fifo_one_at_a_time": {k: fst[k] for k in keys}})
    return out


def config_leg(name: str, steps: int, warmup: int, opts: dict, threads: int) -> dict:
    """One configuration timed like the main leg (build and traversal with
    events over ``steps`` steps after ``warmup``), then checked and timed
    against the oracle on the host: every count, the rows of up to 2000
    particles (all rows for small systems), band pairs of every row, and the
    oracle's own time (cell list on all ``threads`` host threads; for
    N <= 50000 also brute force on one thread and on all threads).  A
    one-type configuration is also timed with the grid comparator."""
    import torch
    import oracle
    import paper_1901_08088_amd as Q
    wl = WORKLOADS[name]
    cfg = make_config(wl)
    n, max_nbr = cfg.n, wl["max_nbr"]
    pos = torch.from_numpy(cfg.pos).cuda()
    types = None if cfg.types is None else torch.from_numpy(cfg.types).cuda()
    nbr = torch.empty((n, max_nbr), dtype=torch.int32, device="cuda")
    cnt = torch.empty(n, dtype=torch.int32, device="cuda")
    ovf = torch.empty(1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    tree = Q.qbvh_build(pos, types, cfg.box, cfg.ntypes, opts)
    for _ in range(warmup):
        Q.qbvh_build(pos, types, cfg.box, cfg.ntypes, opts, tree=tree)
        Q.nlist_build(tree, cfg.rcut, cfg.skin, max_nbr, nbr, cnt, ovf)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e in ev:
        e[0].record(stream)
        Q.qbvh_build(pos, types, cfg.box, cfg.ntypes, opts, tree=tree)
        e[1].record(stream)
        Q.nlist_build(tree, cfg.rcut, cfg.skin, max_nbr, nbr, cnt, ovf)
        e[2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    build_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in ev]))
    trav_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in ev]))
    g_cnt = cnt.cpu().numpy().astype(np.int64)
    pairs = int(g_cnt.sum())
    info = Q.qbvh_info(tree)
    tbytes = traversal_bytes(n, info["nrecords"], int(np.minimum(g_cnt, max_nbr).sum()))
    out = {"workload": describe(wl, cfg), "n": n, "opts": opts, "steps": steps, "build_ms": build_ms,
           "traverse_ms": trav_ms, "ms_per_step": wall * 1e3 / steps, "builds_per_s": steps / wall,
           "directed_pairs": pairs, "pairs_per_s": pairs * steps / wall, "overflow": int(ovf.item()),
           "traversal_algorithmic_gbs": tbytes / (trav_ms * 1e-3) / 1e9,
           "traversal_hbm_frac": tbytes / (trav_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    # the oracle: counts of every row (timed), rows of a sample, band pairs
    t0 = time.perf_counter()
    o_cnt = oracle.neighbor_counts(cfg.pos, cfg.box, cfg.rcut, cfg.skin, types=cfg.types, method="cells",
                                   nthreads=threads)
    out["oracle_cells_all_threads_s"] = time.perf_counter() - t0
    out["count_mismatch_rows"] = int(np.count_nonzero(o_cnt != g_cnt))
    if n <= 50_000:
        # (the thread count is passed on every call: a call sets the pool size)
        for label, nt in (("oracle_brute_1_thread_s", 1), ("oracle_brute_all_threads_s", threads)):
            t0 = time.perf_counter()
            oracle.neighbor_counts(cfg.pos, cfg.box, cfg.rcut, cfg.skin, types=cfg.types, method="brute",
                                   nthreads=nt)
            out[label] = time.perf_counter() - t0
    rng = np.random.default_rng(23)
    q = np.arange(n) if n <= 50_000 else np.sort(rng.choice(n, 2000, replace=False))
    rp, cols = oracle.neighbor_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, types=cfg.types, queries=q,
                                     method="cells", nthreads=threads)
    out["rows"] = row_parity(cfg, gpu_rows(nbr, q), g_cnt, max_nbr, q, rp, cols)
    out["band_pairs"] = band_report(cfg, threads=threads)
    if cfg.types is None:
        out["grid_comparator"] = grid_comparator(cfg, pos, max_nbr, 5)
        out["tree_speedup"] = out["grid_comparator"]["ms"] / out["ms_per_step"]
    log(f"{name}: {out}")
    Q.qbvh_free(tree)
    del nbr
    torch.cuda.empty_cache()
    return out


def cpu_baseline(cfg, sample_rows: int, threads: int):
    """The oracle's cell list timed on this host: three runs, each over the
    rows of a different random sample of ``sample_rows // 3`` particles (the
    binning of all particles included), the median scaled linearly to all
    rows.  Returns the report and the rows of the first sample."""
    import oracle
    n = cfg.n
    per = max(1, min(sample_rows // 3, n))
    times, first = [], None
    for rep in range(3):
        rng = np.random.default_rng(7 + rep)
        q = np.sort(rng.choice(n, per, replace=False)) if per < n else np.arange(n)
        t0 = time.perf_counter()
        rp, cols = oracle.neighbor_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, types=cfg.types, queries=q,
                                         method="cells", nthreads=threads)
        times.append(time.perf_counter() - t0)
        if first is None:
            first = (q, rp, cols)
    dt = float(np.median(times))
    full = dt * n / per
    rep = {"value": 1.0 / full, "unit": "nlist builds/s", "cores": threads, "kind": "oracle",
           "sample": (f"fp64 cell-list oracle on {threads} host threads, median of 3 runs, each over the rows "
                      f"of {per:,} random particles of {n:,} (binning of all {n:,} included; "
                      f"{', '.join(f'{x:.2f}' for x in times)} s), scaled linearly to all rows"),
           "pairs_per_s": float(first[1][-1]) / times[0]}
    return rep, first


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="lj8m", choices=sorted(WORKLOADS))
    ap.add_argument("--leaf-size", type=int, default=BENCH_OPTS["leaf_size"])
    ap.add_argument("--qbits", type=int, default=BENCH_OPTS["qbits"])
    ap.add_argument("--block-size", type=int, default=BENCH_OPTS["block_size"])
    ap.add_argument("--queries-per-wave", type=int, default=0,
                    help="queries sharing one wavefront's walk (0 = chosen from the system size)")
    ap.add_argument("--collapse-radius", type=float, default=0.0,
                    help="subtree collapse by the cost model for this list radius (0 = runs of leaf size)")
    ap.add_argument("--cpu-sample", type=int, default=2_000_000,
                    help="oracle rows timed for the CPU baseline (0 = skip)")
    ap.add_argument("--paper-steps", type=int, default=10,
                    help="traversals timed for the exact-vs-paper-mode comparison (0 = skip)")
    ap.add_argument("--grid-steps", type=int, default=5,
                    help="calls of the grid comparator timed on the same workload (one type only; 0 = skip)")
    ap.add_argument("--f64-steps", type=int, default=10,
                    help="build + traversal steps timed on the same workload as fp64 data (0 = skip)")
    ap.add_argument("--graph-steps", type=int, default=0,
                    help="one-system graph-replayed calls timed on the same workload (0 = skip)")
    ap.add_argument("--batched-steps", type=int, default=20,
                    help="passes timed for the batched-vs-plain ensemble comparison (0 = skip)")
    ap.add_argument("--served-seconds", type=float, default=5.0,
                    help="Poisson-arrival time of the served-stream comparison (0 = skip)")
    ap.add_argument("--config-steps", type=int, default=20,
                    help="steps timed for each of the other configurations (LJ 4000, LJ 1M, colloid 1M, "
                         "WCA 1M, spinodal 1M), each checked against the oracle and, for one type, timed "
                         "against the grid comparator (0 = skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after timing, run a plain copy kernel of this size (counter calibration)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; --gpus must be 1 "
              "(multi-GPU sharding is not implemented)", file=sys.stderr)
        return 2

    import torch
    import paper_1901_08088_amd as Q
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1

    host = host_info()  # before any oracle call: the thread count of the host's pool
    threads = host["oracle_threads"]
    log(f"host: {host}")
    wl = WORKLOADS[args.workload]
    log(f"generating {args.workload}")
    cfg = make_config(wl)
    n, max_nbr = cfg.n, wl["max_nbr"]
    opts = {"leaf_size": args.leaf_size, "qbits": args.qbits, "block_size": args.block_size}
    if args.queries_per_wave:
        opts["queries_per_wave"] = args.queries_per_wave
    if args.collapse_radius > 0:
        opts["collapse_radius"] = args.collapse_radius

    pos = torch.from_numpy(cfg.pos).cuda()
    types = None if cfg.types is None else torch.from_numpy(cfg.types).cuda()
    nbr = torch.empty((n, max_nbr), dtype=torch.int32, device="cuda")
    cnt = torch.empty(n, dtype=torch.int32, device="cuda")
    ovf = torch.empty(1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    tree = Q.qbvh_build(pos, types, cfg.box, cfg.ntypes, opts)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        Q.qbvh_build(pos, types, cfg.box, cfg.ntypes, opts, tree=tree)
        if ev is not None:
            ev[1].record(stream)
        Q.nlist_build(tree, cfg.rcut, cfg.skin, max_nbr, nbr, cnt, ovf)
        if ev is not None:
            ev[2].record(stream)

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    build_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in events]))
    trav_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in events]))
    ms_per_step = wall * 1e3 / args.steps

    counts = cnt.cpu().numpy().astype(np.int64)
    pairs = int(counts.sum())
    stored = int(np.minimum(counts, max_nbr).sum())
    info = Q.qbvh_info(tree)
    tbytes = traversal_bytes(n, info["nrecords"], stored)
    achieved = tbytes / (trav_ms * 1e-3) / 1e9
    builds_per_s = args.steps / wall
    log(f"build {build_ms:.3f} ms, traversal {trav_ms:.3f} ms, {ms_per_step:.3f} ms/step, "
        f"pairs {pairs:,}, overflow {int(ovf.item())}")

    if args.copy_probe_mib > 0:
        copy_probe(args.copy_probe_mib)

    base = parity = None
    if args.cpu_sample > 0:
        log("cpu baseline (oracle) and row parity on its first sample")
        base, (q, rp, cols) = cpu_baseline(cfg, args.cpu_sample, threads)
        parity = {"count_mismatch_rows_in_sample": int(np.count_nonzero(np.diff(rp) != counts[q]))}
        parity.update(row_parity(cfg, gpu_rows(nbr, q), counts, max_nbr, q, rp, cols))
        parity["band_pairs_in_sample"] = band_report(cfg, queries=q, threads=threads)
        del rp, cols
        log(f"parity: {parity}")

    paper = None
    if args.paper_steps > 0 and cfg.types is None:
        log("paper-mode lists (10-bit grid)")
        paper = paper_mode(cfg, pos, args.paper_steps)

    grid = None
    if args.grid_steps > 0 and cfg.types is None:
        log("grid comparator")
        grid = grid_comparator(cfg, pos, max_nbr, args.grid_steps)
        grid["tree_speedup"] = grid["ms"] / ms_per_step
        if grid["directed_pairs"] != pairs:
            raise RuntimeError(f"grid pairs {grid['directed_pairs']} != tree pairs {pairs}")

    f64 = None
    if args.f64_steps > 0:
        log("fp64 particle data")
        f64 = f64_data(cfg, max_nbr, args.f64_steps)

    graph = None
    if args.graph_steps > 0:
        log("one-system graph replay")
        graph = single_graph(cfg, pos, types, max_nbr, args.graph_steps)

    batched = None
    if args.batched_steps > 0:
        log("batched vs plain (ensemble)")
        del nbr
        torch.cuda.empty_cache()
        batched = batched_vs_plain(args.batched_steps)

    serve = None
    if args.served_seconds > 0:
        log("served stream")
        torch.cuda.empty_cache()
        serve = served(args.served_seconds)

    configs = None
    if args.config_steps > 0:
        configs = {}
        for name in ("lj4000", "lj1m", "colloid1m", "wca1m", "spinodal1m"):
            if name == args.workload:
                continue
            log(f"configuration {name}")
            configs[name] = config_leg(name, args.config_steps, max(3, args.warmup // 2), BENCH_OPTS, threads)

    out = {
        "metric": METRIC,
        "value": builds_per_s,
        "unit": "nlist builds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": describe(wl, cfg),
                   "n": n, "max_nbr": max_nbr, "opts": opts, "parallelism": "single GPU"},
        "pairs_per_s": pairs * builds_per_s,
        "directed_pairs": pairs,
        "build_ms": build_ms,
        "traverse_ms": trav_ms,
        "roofline": {"kernel": "k_traverse", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.workload, opts),
                     "traffic_if_reads_scalar": measured_traffic(args.workload, opts, scalar_reads=True),
                     "valu_busy": (TRAFFIC["valu_busy"] if measured_traffic(args.workload, opts) is not None
                                   else None),
                     "algorithmic_bytes": tbytes, "kernel_sources": kernel_source_hash()},
        "cpu_baseline": base,
        "parity": parity,
        "configs": configs,
        "host": host,
        "paper_mode": paper,
        "single_graph": graph,
        "f64_data": f64,
        "grid_comparator": grid,
        "batched": batched,
        "served": serve,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
