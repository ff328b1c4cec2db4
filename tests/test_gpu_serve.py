"""Served form: the continuous-batching server.  Every result is checked
against the oracle; a simulation's rows are bit-identical served alone and
served in a mix of concurrent requests; admission by footprint evicts idle
sessions and refuses what can never fit; per-simulation order is kept."""
import numpy as np
import pytest

import paper_1901_08088_amd as Q
import workloads as W

from nlist_check import compare_rows, require_gpu

pytestmark = pytest.mark.gpu

GiB = 1 << 30


def _submit(srv, c, pos=None, max_nbr=256):
    torch = require_gpu()
    p = torch.from_numpy(np.ascontiguousarray(c.pos if pos is None else pos)).cuda()
    return srv.submit(c.meta.get("sim", 0), p, c.box, c.rcut, c.skin, max_nbr)


def _rows(srv, sim):
    nbr, cnt, ovf = srv.result(sim)
    return nbr.cpu().numpy(), cnt.cpu().numpy(), int(ovf.cpu().item())


def test_server_alone_and_in_the_mix():
    require_gpu()
    sims = W.served_sims(n_sims=24, n_slabs=6, scale=0.01)
    srv = Q.Server(budget_bytes=8 * GiB, max_inflight=2, max_batch=16)
    a = sims[3]
    srv.wait(_submit(srv, a))
    alone = _rows(srv, a.meta["sim"])
    compare_rows(a, *alone, 256)
    tickets = {}
    for c in sims:
        tickets[c.meta["sim"]] = _submit(srv, c)
    for c in sims:
        srv.wait(tickets[c.meta["sim"]])
        print(f"[serve] {c.name} N={c.n}", flush=True)
        got = _rows(srv, c.meta["sim"])
        compare_rows(c, *got, 256)
        if c is a:
            assert np.array_equal(got[1], alone[1]) and np.array_equal(got[0], alone[0]), \
                "rows differ between the request served alone and in the mix"
    st = srv.stats()
    print(f"[serve] stats {st}", flush=True)
    assert st["completed"] == st["submitted"] == len(sims) + 1
    assert st["batches"] < st["completed"]  # requests were batched together
    assert 0 < st["p50_ms"] <= st["p99_ms"]
    srv.close()


def test_server_admission_evicts_and_refuses():
    torch = require_gpu()
    sims = W.served_sims(n_sims=12, n_slabs=3, scale=0.01)
    big = max(c.n for c in sims)
    per = big * 256 * 4 + Q.qbvh_workspace_bytes(big)
    budget = int(3.5 * per)  # room for about three sessions at a time
    srv = Q.Server(budget_bytes=budget, max_inflight=2, max_batch=8)
    huge = torch.zeros((budget // 1024 + 10, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(Q.QbvhError) as e:
        srv.submit(99, huge, (1000.0, 1000.0, 1000.0), [[3.0]], 0.4, 256)
    assert e.value.code == -5  # QBVH_EAGAIN
    for c in sims:
        t = _submit(srv, c)
        srv.wait(t)
        compare_rows(c, *_rows(srv, c.meta["sim"]), 256)
    st = srv.stats()
    assert st["refused"] == 1 and st["completed"] == len(sims)
    assert st["bytes_peak"] <= budget and st["bytes_resident"] <= budget
    srv.close()


def test_server_keeps_per_sim_order():
    require_gpu()
    c = W.served_sims(n_sims=20, n_slabs=4, scale=0.01)[10]
    srv = Q.Server(budget_bytes=4 * GiB, max_inflight=3, max_batch=4)
    rng = np.random.default_rng(3)
    pos = c.pos
    last = None
    tickets = []
    for _ in range(4):
        pos = W.wrap_f32(pos.astype(np.float64) + rng.normal(0.0, 0.05, pos.shape), c.box)
        tickets.append(_submit(srv, c, pos=pos))
        last = pos
    for t in tickets:
        srv.wait(t)
    moved = W.Config(pos=last, box=c.box, rcut=c.rcut, skin=c.skin, name=c.name)
    compare_rows(moved, *_rows(srv, c.meta["sim"]), 256)
    srv.close()
