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

METRIC = "nlist builds/s & pairs/s at 1 GPU vs oracle; batched vs plain; HBM GB/s %"
HBM_PEAK_GBS = 8000.0
BENCH_OPTS = {"leaf_size": 8, "qbits": 16, "block_size": 256}
WORKLOADS = {
    "lj8m": dict(n=8_000_000, rho=0.85, rc=3.0, skin=0.4, max_nbr=256),
    "lj1m": dict(n=1_000_000, rho=0.85, rc=3.0, skin=0.4, max_nbr=256),
    "lj4000": dict(n=4000, rho=0.85, rc=3.0, skin=0.4, max_nbr=256),
}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def traversal_bytes(n: int, nrecords: int, stored_pairs: int) -> int:
    """Algorithmic HBM bytes of one traversal launch: the Z-ordered particle
    array (16 B per particle, queries and candidates alike) read once, every
    record (32 B) and its rope (4 B) read once, every stored neighbor index
    (4 B) and every count (4 B) written once."""
    return 16 * n + 36 * nrecords + 4 * stored_pairs + 4 * n


# HBM traffic of one k_traverse launch on lj8m with BENCH_OPTS, from two rocprofv3
# counter passes (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) divided by the
# factor the same counters read for a plain elementwise copy of known size (the
# --copy-probe-mib kernel).  Valid only for the kernel sources it was taken on:
# ``traffic`` is reported as null once their hash differs.
TRAFFIC = None
KERNEL_SOURCES = ("paper_1901_08088_amd/csrc/traverse.hip", "paper_1901_08088_amd/csrc/qbvh_internal.h")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, opts: dict):
    t = TRAFFIC
    if t is None or t["sources"] != kernel_source_hash() or t["workload"] != workload or t["opts"] != opts:
        return None
    return (t["fetch_kib"] + t["write_kib"]) * 1024.0 / t["copy_factor"]


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


def cpu_baseline(cfg, sample_rows: int) -> dict:
    """The oracle's cell list timed on this host for a bounded sample of rows."""
    import oracle
    n = cfg.n
    rng = np.random.default_rng(7)
    q = np.sort(rng.choice(n, min(sample_rows, n), replace=False)) if sample_rows < n else None
    nq = n if q is None else q.size
    t0 = time.perf_counter()
    rp, _ = oracle.neighbor_lists(cfg.pos, cfg.box, cfg.rcut, cfg.skin, queries=q, method="cells")
    dt = time.perf_counter() - t0
    full = dt * n / nq
    return {"value": 1.0 / full, "unit": "nlist builds/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": (f"fp64 cell-list oracle, rows of {nq:,} of {n:,} particles (binning of all "
                       f"{n:,} included), {dt:.2f} s wall, scaled linearly to all rows"),
            "pairs_per_s": float(rp[-1]) / dt}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="lj8m", choices=sorted(WORKLOADS))
    ap.add_argument("--leaf-size", type=int, default=BENCH_OPTS["leaf_size"])
    ap.add_argument("--qbits", type=int, default=BENCH_OPTS["qbits"])
    ap.add_argument("--block-size", type=int, default=BENCH_OPTS["block_size"])
    ap.add_argument("--cpu-sample", type=int, default=2_000_000,
                    help="oracle rows timed for the CPU baseline (0 = skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after timing, run a plain copy kernel of this size (counter calibration)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1 "
              "(multi-GPU sharding is described in DESIGN.md, not implemented)", file=sys.stderr)
        return 2

    import torch
    import paper_1901_08088_amd as Q
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1

    wl = WORKLOADS[args.workload]
    log(f"generating {args.workload}")
    cfg = W.lj_fluid(wl["n"], rho=wl["rho"], rc=wl["rc"], skin=wl["skin"])
    n, max_nbr = cfg.n, wl["max_nbr"]
    opts = {"leaf_size": args.leaf_size, "qbits": args.qbits, "block_size": args.block_size}

    pos = torch.from_numpy(cfg.pos).cuda()
    nbr = torch.empty((n, max_nbr), dtype=torch.int32, device="cuda")
    cnt = torch.empty(n, dtype=torch.int32, device="cuda")
    ovf = torch.empty(1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    tree = Q.qbvh_build(pos, None, cfg.box, 1, opts)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        Q.qbvh_build(pos, None, cfg.box, 1, opts, tree=tree)
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

    base = None
    if args.cpu_sample > 0:
        log("cpu baseline (oracle)")
        base = cpu_baseline(cfg, args.cpu_sample)

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
        "config": {"workload": f"lj_fluid N={n:,} rho={wl['rho']} rc={wl['rc']} skin={wl['skin']} "
                               f"max_nbr={max_nbr} fp32 (jittered simple-cubic lattice, seed "
                               f"{cfg.meta['seed']})",
                   "n": n, "max_nbr": max_nbr, "opts": opts, "parallelism": "single GPU"},
        "pairs_per_s": pairs * builds_per_s,
        "directed_pairs": pairs,
        "build_ms": build_ms,
        "traverse_ms": trav_ms,
        "roofline": {"kernel": "k_traverse", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(args.workload, opts),
                     "algorithmic_bytes": tbytes, "kernel_sources": kernel_source_hash()},
        "cpu_baseline": base,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
