"""Served form: the continuous-batching server.  Every result is checked
against the oracle; a simulation's rows are bit-identical served alone and
served in a mix of concurrent requests (at test scale and at the stream's full
sizes); admission by footprint evicts idle sessions and refuses what can never
fit; per-simulation order is kept; a leased result is never overwritten."""
import numpy as np
import pytest

import oracle
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
    return srv.read(sim)


def _same_rows(got, ref):
    """The listed entries (row i's first min(count_i, max_nbr)), the counts and
    the flag agree; entries past a row's count are not part of the result (a
    request may be written to a different buffer than the previous one)."""
    (g_nbr, g_cnt, g_ovf), (r_nbr, r_cnt, r_ovf) = got, ref
    if g_ovf != r_ovf or not np.array_equal(g_cnt, r_cnt) or g_nbr.shape != r_nbr.shape:
        return False
    listed = np.arange(g_nbr.shape[1])[None, :] < np.minimum(g_cnt, g_nbr.shape[1])[:, None]
    return np.array_equal(g_nbr[listed], r_nbr[listed])


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
            assert _same_rows(got, alone), "rows differ between the request served alone and in the mix"
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


def test_server_lease_protects_a_result_while_the_next_request_runs():
    # a budget for about two sessions: submitting step k+1 of a sim before its
    # step k is read, with other sims competing for memory, must neither
    # overwrite nor free the leased step-k buffers
    torch = require_gpu()
    sims = W.served_sims(n_sims=10, n_slabs=3, scale=0.01)
    big = max(c.n for c in sims)
    budget = int(2.6 * (big * 256 * 4 + Q.qbvh_workspace_bytes(big)))
    srv = Q.Server(budget_bytes=budget, max_inflight=2, max_batch=4)
    a = sims[4]
    srv.wait(_submit(srv, a))
    lease = srv.result(a.meta["sim"])
    k_nbr = lease.nbr.clone()
    k_cnt = lease.count.clone()
    rng = np.random.default_rng(5)
    moved = W.wrap_f32(a.pos.astype(np.float64) + rng.normal(0.0, 0.3, a.pos.shape), a.box)
    t_next = _submit(srv, a, pos=moved)
    others = [_submit(srv, c) for c in sims if c is not a]
    srv.wait(t_next)
    for t in others:
        srv.wait(t)
    torch.cuda.synchronize()
    # the leased step-k buffers still hold step k, bit for bit
    assert torch.equal(lease.count, k_cnt) and torch.equal(lease.nbr, k_nbr)
    compare_rows(a, lease.nbr.cpu().numpy(), lease.count.cpu().numpy(), int(lease.overflow.cpu().item()), 256)
    lease.release()
    # the published result is step k+1
    cfg = W.Config(pos=moved, box=a.box, rcut=a.rcut, skin=a.skin, name=a.name)
    compare_rows(cfg, *_rows(srv, a.meta["sim"]), 256)
    st = srv.stats()
    assert st["bytes_peak"] <= budget
    srv.close()


def _largest(sims, kind):
    return max((c for c in sims if kind in c.name), key=lambda c: c.n)


@pytest.mark.timeout(900)
def test_server_full_size_alone_and_in_the_mix():
    # the served stream at its stated sizes: the largest slab (60 x 60 x 240) and
    # the largest LJ fluid of the 64 simulations, served alone and then in a mix
    # with 14 other members of the stream; every count against the oracle,
    # 2000 sampled rows exact, and the rows bit-identical alone and in the mix
    torch = require_gpu()
    sims = W.served_sims()
    targets = [_largest(sims, "slab"), _largest(sims, "_lj_")]
    rest = sorted((c for c in sims if all(c is not t for t in targets)), key=lambda c: c.n)[::4][:14]
    srv = Q.Server(budget_bytes=96 * GiB, max_inflight=2, max_batch=16)
    alone = {}
    for c in targets:
        print(f"[serve] alone {c.name} N={c.n}", flush=True)
        srv.wait(_submit(srv, c))
        alone[c.meta["sim"]] = _rows(srv, c.meta["sim"])
    tickets = {c.meta["sim"]: _submit(srv, c) for c in rest[:7] + targets + rest[7:]}
    for sim, t in tickets.items():
        srv.wait(t)
    rng = np.random.default_rng(17)
    for c in targets:
        nbr, cnt, ovf = _rows(srv, c.meta["sim"])
        assert _same_rows((nbr, cnt, ovf), alone[c.meta["sim"]]), \
            f"{c.name}: rows differ between the request served alone and in the mix"
        ocnt = oracle.neighbor_counts(c.pos, c.box, c.rcut, c.skin)
        assert np.array_equal(cnt.astype(np.int64), ocnt), f"{c.name}: counts differ from the oracle"
        assert ovf == int((ocnt > 256).any())
        face = np.min(np.minimum(c.pos, c.box - c.pos), axis=1)
        q = np.unique(np.concatenate([rng.choice(c.n, 1700, replace=False), np.argsort(face)[:300]]))
        compare_rows(c, nbr, cnt, ovf, 256, queries=q)
        print(f"[serve] {c.name} N={c.n}: {int(cnt.sum())} pairs, counts and {q.size} rows match", flush=True)
    for c in rest:
        nbr, cnt, ovf = _rows(srv, c.meta["sim"])
        ocnt = oracle.neighbor_counts(c.pos, c.box, c.rcut, c.skin)
        assert np.array_equal(cnt.astype(np.int64), ocnt), f"{c.name}: counts differ from the oracle"
    st = srv.stats()
    print(f"[serve] stats {st}", flush=True)
    assert st["completed"] == st["submitted"] == len(tickets) + len(targets)
    srv.close()
