"""nlist_build_noalloc: the build + list call on the library's fixed workspace
gives, entry for entry, what qbvh_build + nlist_build give on the same inputs;
two calls in a row (the second smaller, so the workspace holds the first
call's larger tree) and a two-type system; sizes past the fixed workspace are
refused before anything runs."""
import ctypes

import numpy as np
import pytest

import paper_1901_08088_amd as Q
import workloads as W
from paper_1901_08088_amd import capi

from nlist_check import compare_rows, require_gpu, to_dev

pytestmark = pytest.mark.gpu


def _outputs(n, max_nbr, fill):
    torch = require_gpu()
    nbr = torch.full((max(n, 1), max_nbr), fill, dtype=torch.int32, device="cuda")
    cnt = torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda")
    ovf = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    return nbr, cnt, ovf


def _host(nbr, cnt, ovf, n):
    return nbr.cpu().numpy()[:n], cnt.cpu().numpy()[:n], int(ovf.item())


def _plain(cfg, max_nbr, opts):
    """The existing entry points on the same inputs and equally filled outputs."""
    torch = require_gpu()
    pos, types = to_dev(cfg)
    tree = Q.qbvh_build(pos, types, cfg.box, cfg.ntypes, opts)
    nbr, cnt, ovf = _outputs(cfg.n, max_nbr, -7)
    Q.nlist_build(tree, cfg.rcut, cfg.skin, max_nbr, nbr, cnt, ovf)
    torch.cuda.synchronize()
    out = _host(nbr, cnt, ovf, cfg.n)
    Q.qbvh_free(tree)
    return out


def _noalloc(cfg, max_nbr, opts):
    """nlist_build_noalloc called through the raw C interface."""
    torch = require_gpu()
    pos, types = to_dev(cfg)
    nbr, cnt, ovf = _outputs(cfg.n, max_nbr, -7)
    L = capi.lib()
    b = (ctypes.c_float * 3)(*[float(x) for x in np.asarray(cfg.box, np.float32)])
    o = capi._opts(opts)
    rc = np.ascontiguousarray(np.asarray(cfg.rcut, np.float32).reshape(cfg.ntypes, cfg.ntypes))
    code = L.nlist_build_noalloc(ctypes.c_void_p(pos.data_ptr()),
                                 ctypes.c_void_p(types.data_ptr()) if types is not None else None,
                                 cfg.n, cfg.ntypes, b, ctypes.byref(o) if o is not None else None,
                                 rc.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), float(cfg.skin), max_nbr,
                                 ctypes.c_void_p(nbr.data_ptr()), ctypes.c_void_p(cnt.data_ptr()),
                                 ctypes.c_void_p(ovf.data_ptr()),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert code == capi.OK, Q.qbvh_strerror(code)
    torch.cuda.synchronize()
    return _host(nbr, cnt, ovf, cfg.n)


def _same(a, b):
    (an, ac, ao), (bn, bc, bo) = a, b
    return ao == bo and np.array_equal(ac, bc) and np.array_equal(an, bn)


def _two_types(n, seed):
    pos, box = W.uniform(n, [16.0, 16.0, 16.0], seed=seed)
    types = (np.arange(n) % 5 == 0).astype(np.int32)
    rcut = np.array([[1.2, 2.0], [2.0, 2.6]], np.float32)
    return W.Config(pos=pos, box=box, rcut=rcut, skin=0.3, types=types, name=f"two_types_N{n}")


@pytest.mark.parametrize("first,second,max_nbr,opts", [
    (lambda: W.lj_fluid(30000, seed=30000, rho=0.85), lambda: W.lj_fluid(4000), 256, None),
    (lambda: _two_types(12000, 5), lambda: _two_types(777, 6), 128, {"leaf_size": 4, "validate": 1}),
    (lambda: W.lj_fluid(40000, seed=40000, rho=0.85), lambda: W.lj_fluid(12411, seed=12411), 100,
     {"leaf_size": 8, "qbits": 12, "block_size": 128}),
])
def test_noalloc_equals_build_and_list_twice(first, second, max_nbr, opts):
    for make in (first, second):
        cfg = make()
        print(f"[noalloc] {cfg.name} N={cfg.n} max_nbr={max_nbr} opts={opts}", flush=True)
        got = _noalloc(cfg, max_nbr, opts)
        ref = _plain(cfg, max_nbr, opts)
        assert _same(got, ref), f"{cfg.name}: nlist_build_noalloc differs from qbvh_build + nlist_build"
        compare_rows(cfg, *got, max_nbr, queries=np.arange(0, cfg.n, 7))


def test_noalloc_repeat_and_empty():
    cfg = W.lj_fluid(4000)
    a = _noalloc(cfg, 256, None)
    empty = W.Config(pos=np.zeros((0, 3), np.float32), box=cfg.box, rcut=cfg.rcut, skin=cfg.skin, name="empty")
    _noalloc(empty, 256, None)
    b = _noalloc(cfg, 256, None)
    assert _same(a, b)


def test_noalloc_refuses_sizes_past_the_workspace():
    torch = require_gpu()
    n = 1
    while Q.qbvh_workspace_bytes(n) <= Q.NOALLOC_BYTES:
        n *= 2
    lo, hi = n // 2, n  # largest accepted size in [lo, hi)
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if Q.qbvh_workspace_bytes(mid) <= Q.NOALLOC_BYTES:
            lo = mid
        else:
            hi = mid
    assert lo > 1_000_000
    box = (200.0, 200.0, 200.0)
    pos = torch.rand((hi, 3), device="cuda") * 199.0
    nbr, cnt, ovf = _outputs(hi, 4, 5)
    with pytest.raises(Q.QbvhError) as e:
        Q.nlist_build_noalloc(pos, None, box, 1, [[1.0]], 0.2, 4, nbr, cnt, ovf)
    assert e.value.code == Q.ENOSPACE
    torch.cuda.synchronize()
    # nothing was launched: the outputs keep their fill
    assert int(ovf.item()) == -1 and bool((cnt == -1).all().item()) and bool((nbr == 5).all().item())
    # the largest accepted size still runs
    cfg = W.lj_fluid(lo, seed=lo, rho=0.85)
    got = _noalloc(cfg, 256, None)
    assert got[2] == 0
    compare_rows(cfg, *got, 256, queries=np.arange(0, cfg.n, 997))
