"""ctypes binding of ``libqbvh.so`` (the C interface declared in include/qbvh.h).

Argument marshalling only: torch tensors become device pointers, the current
torch stream becomes the hipStream_t, and negative return codes become
``QbvhError``.  Every step of the neighbor search runs in the library's HIP
kernels; there is no fallback.  If the library is missing this module raises
when it is first used.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqbvh.so")

MAX_TYPES = 4
OK, EINVAL, EGEOM, ENOMEM, EHIP, EAGAIN, ENOTSUP, ENOSPACE = 0, -1, -2, -3, -4, -5, -6, -7
NOALLOC_BYTES = 160 << 20  # QBVH_NOALLOC_BYTES
EXPORT = dict(keys=1, perm=2, sorted=3, left=4, right=5, range_f=6, range_l=7, parent=8,
              leaf_parent=9, box_lo=10, box_hi=11, records=12, ropes=13)

C_API = ("qbvh_build", "qbvh_build_f64", "nlist_build", "nlist_build_ex", "nlist_build_many", "nlist_batch_stats", "nlist_batch_release",
         "qbvh_server_create", "qbvh_server_submit", "qbvh_server_poll", "qbvh_server_wait",
         "qbvh_server_result", "qbvh_server_release", "qbvh_server_stats", "qbvh_server_destroy",
         "qbvh_free", "qbvh_strerror", "qbvh_last_hip_error", "qbvh_workspace_bytes", "qbvh_info",
         "qbvh_export", "nlist_build_grid", "qgrid_free", "nlist_build_noalloc")


class QbvhError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = qbvh_strerror(code)
        if code == EHIP:
            msg += f" (hipError {lib().qbvh_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{code}]")


class QbvhOpts(ctypes.Structure):
    _fields_ = [("leaf_size", ctypes.c_int32), ("qbits", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("validate", ctypes.c_int32),
                ("collapse_radius", ctypes.c_float), ("queries_per_wave", ctypes.c_int32)]


class QbvhBatchOpts(ctypes.Structure):
    _fields_ = [("leaf_size", ctypes.c_int32), ("qbits", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("eager", ctypes.c_int32)]


class QbvhBatchStats(ctypes.Structure):
    _fields_ = [("tuned", ctypes.c_int32), ("leaf_size", ctypes.c_int32), ("qbits", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("candidates", ctypes.c_int32),
                ("graphs_captured", ctypes.c_int32), ("calls", ctypes.c_int64), ("best_ms", ctypes.c_float)]


class QbvhServerOpts(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("max_inflight", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("batch", QbvhBatchOpts)]


class QbvhRequest(ctypes.Structure):
    _fields_ = [("sim_id", ctypes.c_int32), ("d_pos", ctypes.c_void_p), ("d_type", ctypes.c_void_p),
                ("n", ctypes.c_int32), ("ntypes", ctypes.c_int32), ("box", ctypes.c_float * 3),
                ("rcut", ctypes.c_void_p), ("skin", ctypes.c_float), ("max_nbr", ctypes.c_int32)]


class QbvhServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("refused", ctypes.c_int64), ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("requests_per_s", ctypes.c_double),
                ("particles_per_s", ctypes.c_double), ("mean_batch", ctypes.c_double),
                ("bytes_resident", ctypes.c_size_t), ("bytes_peak", ctypes.c_size_t)]


class QbvhSystem(ctypes.Structure):
    _fields_ = [("d_pos", ctypes.c_void_p), ("d_type", ctypes.c_void_p), ("n", ctypes.c_int32),
                ("ntypes", ctypes.c_int32), ("box", ctypes.c_float * 3), ("rcut", ctypes.c_void_p),
                ("skin", ctypes.c_float), ("max_nbr", ctypes.c_int32), ("d_nbr", ctypes.c_void_p),
                ("d_count", ctypes.c_void_p), ("d_overflow", ctypes.c_void_p)]


class QbvhInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("ntypes", ctypes.c_int32), ("nrecords", ctypes.c_int32),
                ("leaf_size", ctypes.c_int32), ("qbits", ctypes.c_int32),
                ("tree_start", ctypes.c_int32 * MAX_TYPES), ("tree_count", ctypes.c_int32 * MAX_TYPES),
                ("tree_root", ctypes.c_int32 * MAX_TYPES), ("tree_end", ctypes.c_int32 * MAX_TYPES),
                ("root_lo", (ctypes.c_float * 3) * MAX_TYPES), ("root_hi", (ctypes.c_float * 3) * MAX_TYPES),
                ("h", ctypes.c_double * MAX_TYPES)]


_lib = None
_lock = threading.Lock()


def lib():
    """Load libqbvh.so once; raise if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                                   "`python -m paper_1901_08088_amd.build_ext` (hipcc, gfx950)")
            L = ctypes.CDLL(LIB_PATH)
            P, I32 = ctypes.c_void_p, ctypes.c_int32
            L.qbvh_build.argtypes = [ctypes.POINTER(P), P, P, I32, I32, ctypes.POINTER(ctypes.c_float),
                                     ctypes.POINTER(QbvhOpts), P]
            L.qbvh_build.restype = ctypes.c_int
            L.qbvh_build_f64.argtypes = [ctypes.POINTER(P), P, P, I32, I32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(QbvhOpts), P]
            L.qbvh_build_f64.restype = ctypes.c_int
            L.nlist_build_grid.argtypes = [ctypes.POINTER(P), P, I32, ctypes.POINTER(ctypes.c_float), ctypes.c_float,
                                           ctypes.c_float, I32, I32, P, P, P, P]
            L.nlist_build_grid.restype = ctypes.c_int
            L.qgrid_free.argtypes = [P]
            L.qgrid_free.restype = None
            L.nlist_build.argtypes = [P, ctypes.POINTER(ctypes.c_float), ctypes.c_float, I32, P, P, P, P]
            L.nlist_build.restype = ctypes.c_int
            L.nlist_build_ex.argtypes = [P, ctypes.POINTER(ctypes.c_float), ctypes.c_float, I32, I32, P, P, P, P]
            L.nlist_build_ex.restype = ctypes.c_int
            L.nlist_build_noalloc.argtypes = [P, P, I32, I32, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(QbvhOpts),
                                              ctypes.POINTER(ctypes.c_float), ctypes.c_float, I32, P, P, P, P]
            L.nlist_build_noalloc.restype = ctypes.c_int
            L.nlist_build_many.argtypes = [I32, ctypes.POINTER(QbvhSystem), ctypes.POINTER(QbvhBatchOpts), P]
            L.nlist_build_many.restype = ctypes.c_int
            L.nlist_batch_stats.argtypes = [P, ctypes.POINTER(QbvhBatchStats)]
            L.nlist_batch_stats.restype = ctypes.c_int
            L.nlist_batch_release.argtypes = [P]
            L.nlist_batch_release.restype = None
            L.qbvh_server_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(QbvhServerOpts)]
            L.qbvh_server_create.restype = ctypes.c_int
            L.qbvh_server_submit.argtypes = [P, ctypes.POINTER(QbvhRequest), ctypes.POINTER(ctypes.c_int64)]
            L.qbvh_server_submit.restype = ctypes.c_int
            L.qbvh_server_poll.argtypes = [P, ctypes.c_int64, ctypes.POINTER(I32)]
            L.qbvh_server_poll.restype = ctypes.c_int
            L.qbvh_server_wait.argtypes = [P, ctypes.c_int64]
            L.qbvh_server_wait.restype = ctypes.c_int
            L.qbvh_server_result.argtypes = [P, I32, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P),
                                             ctypes.POINTER(I32), ctypes.POINTER(I32)]
            L.qbvh_server_result.restype = ctypes.c_int
            L.qbvh_server_release.argtypes = [P, I32, P]
            L.qbvh_server_release.restype = ctypes.c_int
            L.qbvh_server_stats.argtypes = [P, ctypes.POINTER(QbvhServerStats)]
            L.qbvh_server_stats.restype = ctypes.c_int
            L.qbvh_server_destroy.argtypes = [P]
            L.qbvh_server_destroy.restype = None
            L.qbvh_free.argtypes = [P]
            L.qbvh_free.restype = None
            L.qbvh_strerror.argtypes = [ctypes.c_int]
            L.qbvh_strerror.restype = ctypes.c_char_p
            L.qbvh_last_hip_error.argtypes = []
            L.qbvh_last_hip_error.restype = ctypes.c_int
            L.qbvh_workspace_bytes.argtypes = [I32, I32, ctypes.POINTER(QbvhOpts)]
            L.qbvh_workspace_bytes.restype = ctypes.c_size_t
            L.qbvh_info.argtypes = [P, ctypes.POINTER(QbvhInfo)]
            L.qbvh_info.restype = ctypes.c_int
            L.qbvh_export.argtypes = [P, I32, P, ctypes.c_size_t, P]
            L.qbvh_export.restype = ctypes.c_int
            _lib = L
    return _lib


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype, name, allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _opts(opts) -> QbvhOpts | None:
    if opts is None:
        return None
    if isinstance(opts, QbvhOpts):
        return opts
    o = QbvhOpts()
    for k, v in dict(opts).items():
        setattr(o, k, float(v) if k == "collapse_radius" else int(v))
    return o


def _check(code: int, where: str):
    if code != OK:
        raise QbvhError(code, where)


class Tree:
    """Owns a ``qbvh_t*``; freed by ``qbvh_free`` or when garbage collected."""

    def __init__(self):
        self.ptr = ctypes.c_void_p(None)
        self.ntypes = 1

    def __del__(self):
        try:
            qbvh_free(self)
        except Exception:
            pass


def qbvh_build(pos, types=None, box=None, ntypes: int = 1, opts=None, tree: Tree | None = None,
               stream=None) -> Tree:
    """Build (or rebuild in place) the quantized BVH of ``pos`` ([n, 3] on the GPU):
    float32 data through qbvh_build, float64 data through qbvh_build_f64 (the
    box is then taken in fp64)."""
    import torch
    t = tree if tree is not None else Tree()
    n = int(pos.shape[0]) if pos is not None else 0
    if pos is not None and (pos.dim() != 2 or pos.shape[1] != 3):
        raise ValueError("pos must have shape [n, 3]")
    f64 = pos is not None and pos.dtype == torch.float64
    pp = _dev_ptr(pos, torch.float64 if f64 else torch.float32, "pos")
    tp = _dev_ptr(types, torch.int32, "types", allow_none=True)
    o = _opts(opts)
    if f64:
        b = (ctypes.c_double * 3)(*[float(x) for x in np.asarray(box, dtype=np.float64).reshape(3)])
        rc = lib().qbvh_build_f64(ctypes.byref(t.ptr), pp, tp, n, int(ntypes), b,
                                  ctypes.byref(o) if o is not None else None, _stream(stream))
    else:
        b = (ctypes.c_float * 3)(*[float(x) for x in np.asarray(box, dtype=np.float32).reshape(3)])
        rc = lib().qbvh_build(ctypes.byref(t.ptr), pp, tp, n, int(ntypes), b,
                              ctypes.byref(o) if o is not None else None, _stream(stream))
    _check(rc, "qbvh_build_f64" if f64 else "qbvh_build")
    t.ntypes = int(ntypes)
    return t


def _rcut_array(rcut, ntypes):
    rc = np.ascontiguousarray(np.asarray(rcut, dtype=np.float32).reshape(ntypes, ntypes))
    return rc, rc.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def nlist_build(tree: Tree, rcut, skin: float, max_nbr: int, nbr, count, overflow, stream=None) -> None:
    """Exact neighbor list of the tree's particles into caller-owned device tensors."""
    import torch
    rc, rp = _rcut_array(rcut, tree.ntypes)
    rc_ = lib().nlist_build(tree.ptr, rp, float(skin), int(max_nbr),
                            _dev_ptr(nbr, torch.int32, "nbr", allow_none=True),
                            _dev_ptr(count, torch.int32, "count"), _dev_ptr(overflow, torch.int32, "overflow"),
                            _stream(stream))
    del rc
    _check(rc_, "nlist_build")


LIST_EXACT, LIST_PAPER = 0, 1


def nlist_build_ex(tree: Tree, rcut, skin: float, max_nbr: int, mode: int, nbr, count, overflow,
                   stream=None) -> None:
    """nlist_build with a list semantics: LIST_EXACT or LIST_PAPER (leaf-box overlap lists)."""
    import torch
    rc, rp = _rcut_array(rcut, tree.ntypes)
    rc_ = lib().nlist_build_ex(tree.ptr, rp, float(skin), int(max_nbr), int(mode),
                               _dev_ptr(nbr, torch.int32, "nbr", allow_none=True),
                               _dev_ptr(count, torch.int32, "count"), _dev_ptr(overflow, torch.int32, "overflow"),
                               _stream(stream))
    del rc
    _check(rc_, "nlist_build_ex")


def nlist_build_noalloc(pos, types, box, ntypes: int, rcut, skin: float, max_nbr: int, nbr, count, overflow,
                        opts=None, stream=None) -> None:
    """qbvh_build + nlist_build in one call on the library's fixed workspace (no allocation)."""
    import torch
    n = int(pos.shape[0]) if pos is not None else 0
    if pos is not None and (pos.dim() != 2 or pos.shape[1] != 3):
        raise ValueError("pos must have shape [n, 3]")
    b = (ctypes.c_float * 3)(*[float(x) for x in np.asarray(box, dtype=np.float32).reshape(3)])
    o = _opts(opts)
    rc, rp = _rcut_array(rcut, int(ntypes))
    rc_ = lib().nlist_build_noalloc(_dev_ptr(pos, torch.float32, "pos", allow_none=True),
                                    _dev_ptr(types, torch.int32, "types", allow_none=True), n, int(ntypes), b,
                                    ctypes.byref(o) if o is not None else None, rp, float(skin), int(max_nbr),
                                    _dev_ptr(nbr, torch.int32, "nbr", allow_none=True),
                                    _dev_ptr(count, torch.int32, "count"),
                                    _dev_ptr(overflow, torch.int32, "overflow"), _stream(stream))
    del rc
    _check(rc_, "nlist_build_noalloc")


def nlist_build_many(systems, opts=None, stream=None) -> None:
    """Batched build + traversal.  ``systems`` is a list of dicts with the keys of qbvh_system_t
    (pos, types, box, rcut, skin, max_nbr, nbr, count, overflow; ntypes optional)."""
    import torch
    arr = (QbvhSystem * max(len(systems), 1))()
    keep = []
    for i, s in enumerate(systems):
        ntypes = int(s.get("ntypes", 1))
        rc, rp = _rcut_array(s["rcut"], ntypes)
        keep.append(rc)
        y = arr[i]
        y.d_pos = _dev_ptr(s["pos"], torch.float32, "pos")
        y.d_type = _dev_ptr(s.get("types"), torch.int32, "types", allow_none=True)
        y.n = int(s["pos"].shape[0])
        y.ntypes = ntypes
        for d, v in enumerate(np.asarray(s["box"], dtype=np.float32).reshape(3)):
            y.box[d] = float(v)
        y.rcut = ctypes.cast(rp, ctypes.c_void_p)
        y.skin = float(s["skin"])
        y.max_nbr = int(s["max_nbr"])
        y.d_nbr = _dev_ptr(s.get("nbr"), torch.int32, "nbr", allow_none=True)
        y.d_count = _dev_ptr(s["count"], torch.int32, "count")
        y.d_overflow = _dev_ptr(s["overflow"], torch.int32, "overflow")
    o = None
    if opts is not None:
        o = QbvhBatchOpts(**{k: int(v) for k, v in dict(opts).items()})
    rc_ = lib().nlist_build_many(len(systems), arr, ctypes.byref(o) if o is not None else None,
                                 _stream(stream))
    del keep
    _check(rc_, "nlist_build_many")


def nlist_batch_stats(stream=None) -> dict:
    """Autotuner state of the last batch shape used on ``stream``."""
    st = QbvhBatchStats()
    _check(lib().nlist_batch_stats(_stream(stream), ctypes.byref(st)), "nlist_batch_stats")
    return {k: getattr(st, k) for k, _ in QbvhBatchStats._fields_}


def nlist_batch_release(stream=None) -> None:
    """Free the batch context of ``stream`` (waits for the stream)."""
    lib().nlist_batch_release(_stream(stream))


class _DeviceArray:
    """A device buffer of the library seen through ``__cuda_array_interface__``
    (torch wraps it without copying)."""

    def __init__(self, ptr: int, shape, typestr: str = "<i4"):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (ptr, False),
                                         "version": 3, "strides": None}


class Server:
    """qbvh_server_*: continuous-batching neighbor-list server (see include/qbvh.h)."""

    def __init__(self, budget_bytes: int, max_inflight: int = 2, max_batch: int = 64, batch_opts=None):
        o = QbvhServerOpts()
        o.budget_bytes = int(budget_bytes)
        o.max_inflight = int(max_inflight)
        o.max_batch = int(max_batch)
        if batch_opts:
            o.batch = QbvhBatchOpts(**{k: int(v) for k, v in dict(batch_opts).items()})
        h = ctypes.c_void_p(None)
        _check(lib().qbvh_server_create(ctypes.byref(h), ctypes.byref(o)), "qbvh_server_create")
        self._h = h
        self._keep = {}

    def submit(self, sim_id: int, pos, box, rcut, skin: float, max_nbr: int, types=None, ntypes: int = 1) -> int:
        """Queue a rebuild of sim ``sim_id`` from device positions ``pos`` [n, 3] (kept alive
        until the request completes); returns the ticket."""
        import torch
        r = QbvhRequest()
        r.sim_id = int(sim_id)
        r.d_pos = _dev_ptr(pos, torch.float32, "pos")
        r.d_type = _dev_ptr(types, torch.int32, "types", allow_none=True)
        r.n = int(pos.shape[0])
        r.ntypes = int(ntypes)
        for d, v in enumerate(np.asarray(box, dtype=np.float32).reshape(3)):
            r.box[d] = float(v)
        rc, rp = _rcut_array(rcut, ntypes)
        r.rcut = ctypes.cast(rp, ctypes.c_void_p)
        r.skin = float(skin)
        r.max_nbr = int(max_nbr)
        t = ctypes.c_int64(0)
        _check(lib().qbvh_server_submit(self._h, ctypes.byref(r), ctypes.byref(t)), "qbvh_server_submit")
        self._keep[t.value] = (pos, types)
        return t.value

    def poll(self, ticket: int) -> bool:
        done = ctypes.c_int32(0)
        _check(lib().qbvh_server_poll(self._h, int(ticket), ctypes.byref(done)), "qbvh_server_poll")
        if done.value:
            self._keep.pop(ticket, None)
        return bool(done.value)

    def wait(self, ticket: int) -> None:
        rc = lib().qbvh_server_wait(self._h, int(ticket))
        self._keep.pop(ticket, None)
        _check(rc, "qbvh_server_wait")

    def result(self, sim_id: int) -> "Lease":
        """Lease the sim's published result: a ``Lease`` whose ``nbr`` [n, max_nbr],
        ``count`` [n] and ``overflow`` [1] device tensors view the session's buffers
        until ``release()`` (also called on leaving a ``with`` block)."""
        import torch
        P = ctypes.c_void_p
        a, b, c = P(None), P(None), P(None)
        n, m = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().qbvh_server_result(self._h, int(sim_id), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                        ctypes.byref(n), ctypes.byref(m)), "qbvh_server_result")
        dev = torch.device("cuda", torch.cuda.current_device())
        nbr = torch.as_tensor(_DeviceArray(a.value, (n.value, m.value)), device=dev)
        cnt = torch.as_tensor(_DeviceArray(b.value, (n.value,)), device=dev)
        ovf = torch.as_tensor(_DeviceArray(c.value, (1,)), device=dev)
        return Lease(self, int(sim_id), a.value, nbr, cnt, ovf)

    def read(self, sim_id: int):
        """Host copies (nbr, count, overflow) of the sim's published result (leased while copying)."""
        import torch
        with self.result(sim_id) as r:
            out = (r.nbr.cpu().numpy(), r.count.cpu().numpy(), int(r.overflow.cpu().item()))
            torch.cuda.synchronize()
        return out

    def stats(self) -> dict:
        st = QbvhServerStats()
        _check(lib().qbvh_server_stats(self._h, ctypes.byref(st)), "qbvh_server_stats")
        return {k: getattr(st, k) for k, _ in QbvhServerStats._fields_}

    def close(self) -> None:
        if self._h is not None and self._h.value:
            lib().qbvh_server_destroy(self._h)
        self._h = None
        self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Lease:
    """One lease on a served result (qbvh_server_result / qbvh_server_release)."""

    def __init__(self, server: Server, sim_id: int, nbr_ptr: int, nbr, count, overflow):
        self._server, self.sim_id, self._ptr = server, sim_id, nbr_ptr
        self.nbr, self.count, self.overflow = nbr, count, overflow

    def release(self) -> None:
        """Return the lease; work that reads the tensors must be finished (or ordered) first."""
        if self._ptr is not None and self._server._h is not None:
            _check(lib().qbvh_server_release(self._server._h, self.sim_id, ctypes.c_void_p(self._ptr)),
                   "qbvh_server_release")
        self._ptr = None
        self.nbr = self.count = self.overflow = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.release()
        return False


def qbvh_free(tree: Tree) -> None:
    if tree is not None and tree.ptr:
        lib().qbvh_free(tree.ptr)
        tree.ptr = ctypes.c_void_p(None)


def qbvh_strerror(code: int) -> str:
    return lib().qbvh_strerror(int(code)).decode()


def qbvh_workspace_bytes(n: int, ntypes: int = 1, opts=None) -> int:
    o = _opts(opts)
    return int(lib().qbvh_workspace_bytes(int(n), int(ntypes), ctypes.byref(o) if o is not None else None))


def qbvh_info(tree: Tree) -> dict:
    """Host summary of a built tree (synchronizes the tree's last stream)."""
    info = QbvhInfo()
    _check(lib().qbvh_info(tree.ptr, ctypes.byref(info)), "qbvh_info")
    nt = info.ntypes
    return dict(n=info.n, ntypes=nt, nrecords=info.nrecords, leaf_size=info.leaf_size, qbits=info.qbits,
                tree_start=list(info.tree_start)[:nt], tree_count=list(info.tree_count)[:nt],
                tree_root=list(info.tree_root)[:nt], tree_end=list(info.tree_end)[:nt],
                root_lo=[list(info.root_lo[t]) for t in range(nt)],
                root_hi=[list(info.root_hi[t]) for t in range(nt)], h=list(info.h)[:nt])


def qbvh_export(tree: Tree, what, dst, stream=None) -> None:
    """Copy an intermediate array of the last build into the device tensor ``dst``."""
    code = EXPORT[what] if isinstance(what, str) else int(what)
    if not dst.is_cuda or not dst.is_contiguous():
        raise ValueError("dst must be a contiguous CUDA tensor")
    nbytes = dst.numel() * dst.element_size()
    _check(lib().qbvh_export(tree.ptr, code, ctypes.c_void_p(dst.data_ptr()), nbytes, _stream(stream)),
           "qbvh_export")


class Grid:
    """Handle of the grid comparator's device workspace (nlist_build_grid)."""

    def __init__(self):
        self.ptr = ctypes.c_void_p()

    def free(self):
        if self.ptr and self.ptr.value:
            lib().qgrid_free(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def nlist_build_grid(pos, box, rcut: float, skin: float, max_nbr: int, nbr, count, overflow,
                     grid: Grid | None = None, stream=None, lanes: int = 0) -> Grid:
    """Exact one-type neighbor lists by the grid method (the comparator of the tree),
    ``lanes`` cooperating lanes per particle (1..32, a power of 2; 0 = 4)."""
    import torch
    g = grid if grid is not None else Grid()
    n = int(pos.shape[0])
    b = (ctypes.c_float * 3)(*[float(x) for x in np.asarray(box, dtype=np.float32).reshape(3)])
    rc = lib().nlist_build_grid(ctypes.byref(g.ptr), _dev_ptr(pos, torch.float32, "pos"), n, b, float(rcut),
                                float(skin), int(lanes), int(max_nbr), _dev_ptr(nbr, torch.int32, "nbr", allow_none=True),
                                _dev_ptr(count, torch.int32, "count"), _dev_ptr(overflow, torch.int32, "overflow"),
                                _stream(stream))
    _check(rc, "nlist_build_grid")
    return g
