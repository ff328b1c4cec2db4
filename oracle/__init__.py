"""CPU oracle for the quantized-BVH neighbor search.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the library under
``paper_1901_08088_amd`` never does, and the two share no code.

``nlist_oracle.c`` evaluates the neighbor sets by definition (fp64 minimum
image distances, inclusive cutoff, self excluded); ``tree.py`` writes out, step
by step, the tree the method builds (Morton codes, stable sort, radix tree,
bottom-up boxes, quantized preorder layout) so that each build step of the GPU
path can be compared with it bit for bit.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nlist_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()


def build(force: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc (fp64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-std=c11", "-Wall", "-Wextra", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def configure(lib):
    """Declare the C signatures on a loaded oracle library (also used for test variants)."""
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    I32 = ctypes.c_int32
    for name in ("oracle_count_brute", "oracle_count_cells"):
        f = getattr(lib, name)
        f.argtypes = [I64, P, P, I32, P, P, I64, P, P, ctypes.c_int]
        f.restype = ctypes.c_int
    for name in ("oracle_fill_brute", "oracle_fill_cells"):
        f = getattr(lib, name)
        f.argtypes = [I64, P, P, I32, P, P, I64, P, P, P, ctypes.c_int]
        f.restype = ctypes.c_int
    lib.oracle_pair_d2.argtypes = [P, P, P]
    lib.oracle_pair_d2.restype = ctypes.c_double
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = ctypes.c_int
    lib.oracle_band_count.argtypes = [I64, P, P, I32, P, P, I64, P, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int, P, P, ctypes.c_int]
    lib.oracle_band_count.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            _lib = configure(ctypes.CDLL(_LIB_PATH))
    return _lib


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def rlist2_table(rcut, skin) -> np.ndarray:
    """Squared list radius per type pair, (rc + skin)^2 in fp64 from the fp32 inputs.

    A type pair with rc <= 0 is never listed and gets -1.
    """
    rc = np.asarray(rcut, dtype=np.float32)
    rc = rc.reshape((1, 1)) if rc.ndim == 0 else rc
    r = rc.astype(np.float64) + np.float64(np.float32(skin))
    r2 = r * r
    return np.where(rc > 0, r2, -1.0).astype(np.float64)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _as_f64(pos, box):
    """Positions and box as fp64.  fp32 data (the default) is converted exactly;
    fp64 positions keep their values and take the box as given in fp64."""
    pos = np.asarray(pos)
    if pos.dtype == np.float64:
        return (np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3),
                np.ascontiguousarray(np.asarray(box, dtype=np.float64).reshape(3)))
    return (np.ascontiguousarray(pos, dtype=np.float32).reshape(-1, 3).astype(np.float64),
            np.ascontiguousarray(np.asarray(box, dtype=np.float32).astype(np.float64).reshape(3)))


def _prep(pos, box, rcut, skin, types):
    pos, box = _as_f64(pos, box)
    r2 = np.ascontiguousarray(rlist2_table(rcut, skin))
    ntypes = r2.shape[0]
    t = None if types is None else np.ascontiguousarray(types, dtype=np.int32)
    return pos, box, r2, ntypes, t


def neighbor_lists(pos, box, rcut, skin, types=None, queries=None, method: str = "auto",
                   nthreads: int = 0):
    """Sorted neighbor rows as CSR ``(row_ptr int64 [nq+1], cols int32)``.

    ``queries`` selects the particles whose rows are returned (default: all,
    in index order).  ``method`` is "brute", "cells" or "auto" (cells unless
    the box is too small for a 3-cell stencil on some axis).
    """
    lib = _load()
    pos, box64, r2, ntypes, t = _prep(pos, box, rcut, skin, types)
    n = pos.shape[0]
    q = None if queries is None else np.ascontiguousarray(queries, dtype=np.int64)
    nq = n if q is None else q.shape[0]
    count = np.zeros(max(nq, 1), dtype=np.int64)
    use_cells = method in ("auto", "cells")
    if use_cells:
        rc = lib.oracle_count_cells(n, _ptr(pos), _ptr(t), ntypes, _ptr(box64), _ptr(r2), nq,
                                    _ptr(q), _ptr(count), nthreads)
        if rc == 1:
            if method == "cells":
                raise ValueError("box too small for a 3x3x3 cell stencil")
            use_cells = False
        elif rc != 0:
            raise RuntimeError("oracle_count_cells failed")
    if not use_cells:
        if lib.oracle_count_brute(n, _ptr(pos), _ptr(t), ntypes, _ptr(box64), _ptr(r2), nq,
                                  _ptr(q), _ptr(count), nthreads) != 0:
            raise RuntimeError("oracle_count_brute failed")
    row_ptr = np.zeros(nq + 1, dtype=np.int64)
    np.cumsum(count[:nq], out=row_ptr[1:])
    cols = np.zeros(max(int(row_ptr[-1]), 1), dtype=np.int32)
    fill = lib.oracle_fill_cells if use_cells else lib.oracle_fill_brute
    if fill(n, _ptr(pos), _ptr(t), ntypes, _ptr(box64), _ptr(r2), nq, _ptr(q), _ptr(row_ptr),
            _ptr(cols), nthreads) != 0:
        raise RuntimeError("oracle fill failed")
    return row_ptr, cols[: int(row_ptr[-1])]


def neighbor_counts(pos, box, rcut, skin, types=None, queries=None, method: str = "auto",
                    nthreads: int = 0) -> np.ndarray:
    """|S_i| for the selected queries (int64)."""
    lib = _load()
    pos, box64, r2, ntypes, t = _prep(pos, box, rcut, skin, types)
    n = pos.shape[0]
    q = None if queries is None else np.ascontiguousarray(queries, dtype=np.int64)
    nq = n if q is None else q.shape[0]
    count = np.zeros(max(nq, 1), dtype=np.int64)
    rc = 1
    if method in ("auto", "cells"):
        rc = lib.oracle_count_cells(n, _ptr(pos), _ptr(t), ntypes, _ptr(box64), _ptr(r2), nq,
                                    _ptr(q), _ptr(count), nthreads)
        if rc == 1 and method == "cells":
            raise ValueError("box too small for a 3x3x3 cell stencil")
        if rc < 0:
            raise RuntimeError("oracle_count_cells failed")
    if rc == 1:
        if lib.oracle_count_brute(n, _ptr(pos), _ptr(t), ntypes, _ptr(box64), _ptr(r2), nq,
                                  _ptr(q), _ptr(count), nthreads) != 0:
            raise RuntimeError("oracle_count_brute failed")
    return count[:nq]


def pair_d2(pi, pj, box) -> float:
    """fp64 minimum-image squared distance of two points (fp32, or fp64 with an
    fp64 box), same arithmetic as the lists."""
    lib = _load()
    ab, L = _as_f64(np.stack([np.asarray(pi), np.asarray(pj)]), box)
    a = np.ascontiguousarray(ab[0])
    b = np.ascontiguousarray(ab[1])
    return float(lib.oracle_pair_d2(_ptr(a), _ptr(b), _ptr(L)))


def band_counts(pos, box, rcut, skin, types=None, queries=None, rel: float = 1e-5,
                abs_tol: float = 1e-5, method: str = "auto", nthreads: int = 0):
    """Per query, the number of partners j != i (listed type pairs only) whose
    fp64 minimum-image distance lies within the band around the list radius r,
    under the two readings of a 1e-5 tolerance: ``|d - r| <= rel * r``
    (relative) and ``|d - r| <= abs_tol`` (absolute, in sigma).

    Both arrays are int64 [nq].  These are the pairs where a distance computed
    in another floating-point order may fall on the other side of eq. (2)'s
    inclusive test.  ``method``: "brute", "cells" or "auto" (cells unless the
    box is too small for a 3-cell stencil at the widened radius).
    """
    lib = _load()
    pos, box64, r2, ntypes, t = _prep(pos, box, rcut, skin, types)
    n = pos.shape[0]
    q = None if queries is None else np.ascontiguousarray(queries, dtype=np.int64)
    nq = n if q is None else q.shape[0]
    a = np.zeros(max(nq, 1), dtype=np.int64)
    b = np.zeros(max(nq, 1), dtype=np.int64)
    rc = 1
    if method in ("auto", "cells"):
        rc = lib.oracle_band_count(n, _ptr(pos), _ptr(t), ntypes, _ptr(box64), _ptr(r2), nq, _ptr(q),
                                   float(rel), float(abs_tol), 1, _ptr(a), _ptr(b), nthreads)
        if rc == 1 and method == "cells":
            raise ValueError("box too small for a 3x3x3 cell stencil")
        if rc < 0:
            raise RuntimeError("oracle_band_count failed")
    if rc == 1:
        if lib.oracle_band_count(n, _ptr(pos), _ptr(t), ntypes, _ptr(box64), _ptr(r2), nq, _ptr(q),
                                 float(rel), float(abs_tol), 0, _ptr(a), _ptr(b), nthreads) != 0:
            raise RuntimeError("oracle_band_count failed")
    return a[:nq], b[:nq]
