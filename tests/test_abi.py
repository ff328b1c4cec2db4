"""The C interface: the library loads, exports every declared symbol, and rejects
bad arguments before touching the device.  Runs without a GPU."""
import ctypes
import os
import re

import pytest

import paper_1901_08088_amd as Q
from paper_1901_08088_amd import capi

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "qbvh.h")


def declared_functions():
    src = open(HEADER).read()
    return re.findall(r"^QBVH_API\s+[\w\s\*]+?\b(\w+)\s*\(", src, flags=re.M)


def test_header_declares_the_interface():
    names = set(declared_functions())
    assert names == set(capi.C_API)


def test_library_exports_every_declared_symbol():
    lib = Q.lib()
    raw = ctypes.CDLL(capi.LIB_PATH)
    for name in declared_functions():
        assert hasattr(raw, name), name
        assert hasattr(lib, name)


def test_strerror_and_codes():
    assert Q.qbvh_strerror(0) == "ok"
    for code in (capi.EINVAL, capi.EGEOM, capi.ENOMEM, capi.EHIP, capi.EAGAIN, capi.ENOTSUP):
        assert Q.qbvh_strerror(code) not in ("ok", "unknown error")
    assert Q.qbvh_strerror(12345) == "unknown error"


def test_workspace_bytes():
    a = Q.qbvh_workspace_bytes(1000)
    b = Q.qbvh_workspace_bytes(1_000_000)
    assert 0 < a < b
    assert 100 < b / 1_000_000 < 200  # about 128 bytes per particle
    assert Q.qbvh_workspace_bytes(-1) == 0
    assert Q.qbvh_workspace_bytes(10, ntypes=5) == 0
    assert Q.qbvh_workspace_bytes(10, opts={"leaf_size": 9}) == 0


def _build_rc(n=10, ntypes=1, box=(5.0, 5.0, 5.0), opts=None, pos=1, typ=None, tree_ptr=True):
    lib = Q.lib()
    t = ctypes.c_void_p(None)
    b = (ctypes.c_float * 3)(*box)
    o = capi._opts(opts)
    return lib.qbvh_build(ctypes.byref(t) if tree_ptr else None,
                          ctypes.c_void_p(pos) if pos else None,
                          ctypes.c_void_p(typ) if typ else None, n, ntypes, b,
                          ctypes.byref(o) if o is not None else None, None)


@pytest.mark.parametrize("kwargs", [
    dict(tree_ptr=False),
    dict(n=-1),
    dict(ntypes=0),
    dict(ntypes=5),
    dict(box=(5.0, 0.0, 5.0)),
    dict(box=(5.0, float("nan"), 5.0)),
    dict(box=(float("inf"), 5.0, 5.0)),
    dict(pos=0),
    dict(ntypes=2, typ=None),
    dict(opts={"leaf_size": 9}),
    dict(opts={"leaf_size": -1}),
    dict(opts={"qbits": 7}),
    dict(opts={"qbits": 17}),
    dict(opts={"block_size": 96}),
    dict(opts={"block_size": 512}),
    dict(opts={"block_size": 1024}),
    dict(opts={"validate": 2}),
])
def test_build_rejects_bad_arguments_without_device_work(kwargs):
    assert _build_rc(**kwargs) == capi.EINVAL


def test_nlist_rejects_null_tree():
    lib = Q.lib()
    rc = (ctypes.c_float * 1)(3.0)
    flag = ctypes.c_int32(0)
    assert lib.nlist_build(None, rc, 0.4, 16, None, None, ctypes.byref(flag), None) == capi.EINVAL


def test_batch_rejects_bad_counts():
    lib = Q.lib()
    assert lib.nlist_build_many(-1, None, None, None) == capi.EINVAL
    assert lib.nlist_build_many(3, None, None, None) == capi.EINVAL


def test_package_does_not_import_the_oracle():
    pkg = os.path.dirname(Q.__file__)
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert not re.search(r"^\s*(import|from)\s+oracle\b", src, flags=re.M), fn
