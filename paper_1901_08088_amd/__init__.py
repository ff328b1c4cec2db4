"""Quantized-BVH neighbor lists for AMD Instinct MI355X (gfx950).

The neighbor search runs in hand-written HIP kernels behind the C interface
declared in ``include/qbvh.h`` (``libqbvh.so``, built in-tree by
``build_ext.py``).  ``capi`` is a thin ctypes binding with the same names.
The library is loaded on first use, not at import.
"""
from .capi import (EINVAL, ENOSPACE, ENOTSUP, EXPORT, LIST_EXACT, LIST_PAPER, NOALLOC_BYTES, Grid, Lease,  # noqa: F401
                   QbvhError, QbvhOpts, Server, Tree, lib, nlist_batch_release, nlist_batch_stats, nlist_build,
                   nlist_build_ex, nlist_build_grid, nlist_build_many, nlist_build_noalloc, qbvh_build, qbvh_export,
                   qbvh_free, qbvh_info, qbvh_strerror, qbvh_workspace_bytes)

__all__ = ["EINVAL", "ENOSPACE", "ENOTSUP", "EXPORT", "Grid", "LIST_EXACT", "LIST_PAPER", "Lease", "NOALLOC_BYTES",
           "QbvhError", "QbvhOpts", "Server", "Tree", "lib", "nlist_batch_release", "nlist_batch_stats",
           "nlist_build", "nlist_build_ex", "nlist_build_grid", "nlist_build_many", "nlist_build_noalloc",
           "qbvh_build", "qbvh_export", "qbvh_free", "qbvh_info", "qbvh_strerror", "qbvh_workspace_bytes"]
